// Spectral-convolution network of the learned warm start (include/stfd_fno.h), FP32.
//
// Every layer is a strided batched GEMM (pointwise channel mixing, truncated DFTs with
// precomputed cos/sin matrices, projection) plus elementwise kernels (GELU, complex
// per-mode mixing, bias, loss, Adam).  Backward passes are the adjoint GEMMs; weight
// gradients over the large row dimension use split-K partial products summed in a fixed
// order, so every result is deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/stfd.h"
#include "../../include/stfd_fno.h"

namespace stfd {
namespace fno {

static thread_local int g_hip_err = 0;
#define FNO_HIP(expr)             \
  do {                            \
    hipError_t e_ = (expr);       \
    if (e_ != hipSuccess) {       \
      g_hip_err = int(e_);        \
      return STFD_EHIP;           \
    }                             \
  } while (0)

// ---------------------------------------------------------------------------
// GEMM: C(m,n) = alpha sum_k A(m,k) B(k,n) + bias(n) + beta C(m,n), per batch b, with
// A(m,k) = A[b sab + m sam + k sak], B(k,n) = B[b sbb + k sbk + n sbn], C(m,n) = C[b scb + m scm + n scn].
// 64 x 64 output tile per 256-thread block, 4 x 4 per thread, K staged through LDS in steps of 16.
// ---------------------------------------------------------------------------
struct GemmArgs {
  int M, N, K;
  const float* A;
  int64_t sam, sak, sab;
  const float* B;
  int64_t sbk, sbn, sbb;
  float* C;
  int64_t scm, scn, scb;
  const float* bias;
  float alpha, beta;
};

__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g) {
  __shared__ float As[16][68];
  __shared__ float Bs[16][68];
  const int b = blockIdx.z;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const float* A = g.A + int64_t(b) * g.sab;
  const float* B = g.B + int64_t(b) * g.sbb;
  float* C = g.C + int64_t(b) * g.scb;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  float acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0f;
  for (int k0 = 0; k0 < g.K; k0 += 16) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = tid + 256 * u;
      const int mm = idx & 63, kk = idx >> 6;
      const int m = m0 + mm, k = k0 + kk;
      As[kk][mm] = (m < g.M && k < g.K) ? A[int64_t(m) * g.sam + int64_t(k) * g.sak] : 0.0f;
      const int n = n0 + mm;
      Bs[kk][mm] = (n < g.N && k < g.K) ? B[int64_t(k) * g.sbk + int64_t(n) * g.sbn] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = As[kk][ty * 4 + i];
        bb[i] = Bs[kk][tx * 4 + i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], bb[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + ty * 4 + i;
    if (m >= g.M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tx * 4 + j;
      if (n >= g.N) continue;
      float v = g.alpha * acc[i][j];
      if (g.bias) v += g.bias[n];
      float* c = C + int64_t(m) * g.scm + int64_t(n) * g.scn;
      if (g.beta != 0.0f) v += g.beta * *c;
      *c = v;
    }
  }
}

// out[i] = sum_c parts[c][i] (fixed order)
__global__ void __launch_bounds__(256) sum_parts_kernel(const float* parts, int nparts, int64_t n, float* out,
                                                        float beta) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    float s = 0.0f;
    for (int c = 0; c < nparts; ++c) s += parts[int64_t(c) * n + i];
    out[i] = (beta != 0.0f) ? s + beta * out[i] : s;
  }
}

// column sums of X [rows][ncol]: partials over row chunks, parts[chunk][col]
__global__ void __launch_bounds__(256) colsum_part_kernel(const float* X, int64_t rows, int ncol, int64_t chunk,
                                                          float* parts) {
  const int col = blockIdx.x * 64 + (threadIdx.x & 63);
  const int grp = threadIdx.x >> 6;
  const int64_t r0 = int64_t(blockIdx.y) * chunk;
  const int64_t r1 = min(rows, r0 + chunk);
  __shared__ float red[4][64];
  float s = 0.0f;
  if (col < ncol)
    for (int64_t r = r0 + grp; r < r1; r += 4) s += X[r * ncol + col];
  red[grp][threadIdx.x & 63] = s;
  __syncthreads();
  if (grp == 0 && col < ncol)
    parts[int64_t(blockIdx.y) * ncol + col] =
        (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

__global__ void __launch_bounds__(256) gelu_kernel(const float* z, float* a, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    a[i] = gelu_f(z[i]);
}

__global__ void __launch_bounds__(256) gelu_bwd_kernel(const float* z, const float* da, float* dz, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    dz[i] = da[i] * gelu_d(z[i]);
}

// Per-mode complex channel mixing.  X, Y layout [b][k2][part][k1][ch]; R layout [k2][k1][c][o].
__global__ void __launch_bounds__(256) mix_fwd_kernel(const float* X, const float* Rr, const float* Ri, float* Y,
                                                      int B, int M1, int M2, int C) {
  const int64_t total = int64_t(B) * M2 * M1 * C;
  for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total; g += int64_t(gridDim.x) * blockDim.x) {
    const int o = int(g % C);
    const int k1 = int((g / C) % M1);
    const int k2 = int((g / (int64_t(C) * M1)) % M2);
    const int b = int(g / (int64_t(C) * M1 * M2));
    const float* xr = X + ((int64_t(b) * M2 + k2) * 2 * M1 + k1) * C;
    const float* xi = xr + int64_t(M1) * C;
    const float* rr = Rr + (int64_t(k2) * M1 + k1) * C * C + o;
    const float* ri = Ri + (int64_t(k2) * M1 + k1) * C * C + o;
    float yr = 0.0f, yi = 0.0f;
    for (int c = 0; c < C; ++c) {
      const float a = xr[c], bb = xi[c], wr = rr[int64_t(c) * C], wi = ri[int64_t(c) * C];
      yr = fmaf(a, wr, fmaf(-bb, wi, yr));
      yi = fmaf(a, wi, fmaf(bb, wr, yi));
    }
    float* y = Y + ((int64_t(b) * M2 + k2) * 2 * M1 + k1) * C + o;
    y[0] = yr;
    y[int64_t(M1) * C] = yi;
  }
}

// dX from dY: dX_r[c] = sum_o dY_r Rr[c,o] + dY_i Ri[c,o],  dX_i[c] = sum_o -dY_r Ri[c,o] + dY_i Rr[c,o]
__global__ void __launch_bounds__(256) mix_bwd_in_kernel(const float* dY, const float* Rr, const float* Ri, float* dX,
                                                         int B, int M1, int M2, int C) {
  const int64_t total = int64_t(B) * M2 * M1 * C;
  for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total; g += int64_t(gridDim.x) * blockDim.x) {
    const int c = int(g % C);
    const int k1 = int((g / C) % M1);
    const int k2 = int((g / (int64_t(C) * M1)) % M2);
    const int b = int(g / (int64_t(C) * M1 * M2));
    const float* dyr = dY + ((int64_t(b) * M2 + k2) * 2 * M1 + k1) * C;
    const float* dyi = dyr + int64_t(M1) * C;
    const float* rr = Rr + ((int64_t(k2) * M1 + k1) * C + c) * C;
    const float* ri = Ri + ((int64_t(k2) * M1 + k1) * C + c) * C;
    float xr = 0.0f, xi = 0.0f;
    for (int o = 0; o < C; ++o) {
      xr = fmaf(dyr[o], rr[o], fmaf(dyi[o], ri[o], xr));
      xi = fmaf(-dyr[o], ri[o], fmaf(dyi[o], rr[o], xi));
    }
    float* dx = dX + ((int64_t(b) * M2 + k2) * 2 * M1 + k1) * C + c;
    dx[0] = xr;
    dx[int64_t(M1) * C] = xi;
  }
}

// dR_r[c,o] = sum_b X_r dY_r + X_i dY_i,  dR_i[c,o] = sum_b X_r dY_i - X_i dY_r
__global__ void __launch_bounds__(256) mix_bwd_w_kernel(const float* X, const float* dY, float* dRr, float* dRi, int B,
                                                        int M1, int M2, int C) {
  const int64_t total = int64_t(M2) * M1 * C * C;
  for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total; g += int64_t(gridDim.x) * blockDim.x) {
    const int o = int(g % C);
    const int c = int((g / C) % C);
    const int k1 = int((g / (int64_t(C) * C)) % M1);
    const int k2 = int(g / (int64_t(C) * C * M1));
    float gr = 0.0f, gi = 0.0f;
    for (int b = 0; b < B; ++b) {
      const int64_t base = ((int64_t(b) * M2 + k2) * 2 * M1 + k1) * C;
      const float xr = X[base + c], xi = X[base + int64_t(M1) * C + c];
      const float yr = dY[base + o], yi = dY[base + int64_t(M1) * C + o];
      gr = fmaf(xr, yr, fmaf(xi, yi, gr));
      gi = fmaf(xr, yi, fmaf(-xi, yr, gi));
    }
    dRr[g] = gr;
    dRi[g] = gi;
  }
}

// relative l2: per-sample partial sums of (y - t)^2 and t^2
__global__ void __launch_bounds__(256) rel_l2_part_kernel(const float* y, const float* t, int64_t n, float* parts) {
  const int b = blockIdx.y;
  __shared__ float red[2][256];
  float se = 0.0f, st = 0.0f;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const float tv = t[int64_t(b) * n + i];
    const float e = y[int64_t(b) * n + i] - tv;
    se = fmaf(e, e, se);
    st = fmaf(tv, tv, st);
  }
  red[0][threadIdx.x] = se;
  red[1][threadIdx.x] = st;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    parts[(int64_t(b) * gridDim.x + blockIdx.x) * 2] = red[0][0];
    parts[(int64_t(b) * gridDim.x + blockIdx.x) * 2 + 1] = red[1][0];
  }
}

// per-sample loss terms and gradient scales (one thread)
__global__ void rel_l2_final_kernel(const float* parts, int nparts, int batch, float* scal) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float loss = 0.0f;
  for (int b = 0; b < batch; ++b) {
    float se = 0.0f, st = 0.0f;
    for (int k = 0; k < nparts; ++k) {
      se += parts[(int64_t(b) * nparts + k) * 2];
      st += parts[(int64_t(b) * nparts + k) * 2 + 1];
    }
    const float e = sqrtf(se), tn = sqrtf(st);
    loss += (tn > 0.0f) ? e / tn : e;
    scal[1 + b] = (e > 0.0f && tn > 0.0f) ? 1.0f / (float(batch) * e * tn) : 0.0f;
  }
  scal[0] = loss / float(batch);
}

__global__ void __launch_bounds__(256) rel_l2_grad_kernel(const float* y, const float* t, const float* scal, int64_t n,
                                                          float* dy) {
  const int b = blockIdx.y;
  const float s = scal[1 + b];
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    dy[int64_t(b) * n + i] = s * (y[int64_t(b) * n + i] - t[int64_t(b) * n + i]);
}

__global__ void __launch_bounds__(256) adam_kernel(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                                                   float b1, float b2, float eps, float bc1, float bc2) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
}

__global__ void __launch_bounds__(256) to_f64_kernel(const float* y, double* x, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    x[i] = double(y[i]);
}

// e = y - t (t may be nullptr) in FP64
__global__ void __launch_bounds__(256) diff_f64_kernel(const float* y, const float* t, double* e, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    e[i] = double(y[i]) - (t ? double(t[i]) : 0.0);
}

// per-sample partial sums of e . Ae (FP64)
__global__ void __launch_bounds__(256) energy_part_kernel(const double* e, const double* Ae, int64_t n,
                                                          double* parts) {
  const int b = blockIdx.y;
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    s = fma(e[int64_t(b) * n + i], Ae[int64_t(b) * n + i], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) parts[int64_t(b) * gridDim.x + blockIdx.x] = red[0];
}

// per-sample energies, loss (1/B) sum_b sqrt(E_b / T_b) and gradient scales (one thread)
__global__ void energy_final_kernel(const double* parts, int nparts, int batch, const double* t_energy,
                                    double* scal) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double loss = 0.0;
  for (int b = 0; b < batch; ++b) {
    double E = 0.0;
    for (int k = 0; k < nparts; ++k) E += parts[int64_t(b) * nparts + k];
    scal[2 + batch + b] = E;
    const double T = t_energy ? t_energy[b] : 1.0;
    const double rel = (E > 0.0 && T > 0.0) ? sqrt(E / T) : 0.0;
    loss += rel;
    // d sqrt(e^H A e / T) / de = A e / sqrt(E T)
    scal[2 + b] = (E > 0.0 && T > 0.0) ? 1.0 / (double(batch) * sqrt(E * T)) : 0.0;
  }
  scal[0] = loss / double(batch);
}

__global__ void __launch_bounds__(256) energy_grad_kernel(const double* Ae, const double* scal, int64_t n, float* dy) {
  const int b = blockIdx.y;
  const double s = scal[2 + b];
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    dy[int64_t(b) * n + i] = float(s * Ae[int64_t(b) * n + i]);
}

inline int grid_for(int64_t n) { return int(std::min<int64_t>((n + 255) / 256, 16384)); }

}  // namespace fno
}  // namespace stfd

using namespace stfd::fno;

struct stfd_fno {
  stfd_fno_desc d;
  int64_t nparams = 0;
  float* params = nullptr;
  float* grads = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  int step = 0;
  // parameter offsets
  int64_t oWp, obp, oQ1, oq1, oQ2, oq2;
  std::vector<int64_t> oW, ob, oRr, oRi;
  // DFT matrices
  float* D1 = nullptr;  // [2 M1][W]  forward along i_1, rows (part, k1)
  float* D2 = nullptr;  // [2 M2][2 H] forward along i_2, rows (k2, part), cols (i2, part)
  float* E2 = nullptr;  // [2 H][2 M2] inverse along i_2
  float* E1 = nullptr;  // [W][2 M1]   inverse along i_1 (half-spectrum weights and 1/(HW))
  // activations of the last forward
  float* x = nullptr;                // [B][H][W][c_in]
  std::vector<float*> a, z, Xs;      // a_l, z_l ([B HW C]), X_l ([B][2 M2][M1][C])
  float *F1 = nullptr, *Ybuf = nullptr, *T2 = nullptr;
  float *p1 = nullptr, *g1 = nullptr;  // [B HW proj]
  // backward scratch
  float *da = nullptr, *dz = nullptr, *dp = nullptr, *dX = nullptr, *parts = nullptr;
  int64_t parts_n = 0;
  float* scal = nullptr;  // loss scratch
  int last_batch = 0;
  std::vector<void*> allocs;
};

namespace {

int gemm(hipStream_t s, int batch, int M, int N, int K, const float* A, int64_t sam, int64_t sak, int64_t sab,
         const float* B, int64_t sbk, int64_t sbn, int64_t sbb, float* C, int64_t scm, int64_t scn, int64_t scb,
         const float* bias, float alpha, float beta) {
  if (M <= 0 || N <= 0 || batch <= 0) return STFD_OK;
  GemmArgs g{M, N, K, A, sam, sak, sab, B, sbk, sbn, sbb, C, scm, scn, scb, bias, alpha, beta};
  dim3 grid(unsigned((N + 63) / 64), unsigned((M + 63) / 64), unsigned(batch));
  hipLaunchKernelGGL(gemm_kernel, grid, dim3(256), 0, s, g);
  FNO_HIP(hipGetLastError());
  return STFD_OK;
}

// Weight gradient C[M][N] = A^T B with A [rows][M], B [rows][N] (row-major), rows large:
// split-K into chunks of partial products, summed in chunk order.
int wgrad(stfd_fno* net, hipStream_t s, int64_t rows, int M, int N, const float* A, const float* B, float* C) {
  const int64_t chunk = 2048;
  const int64_t nfull = rows / chunk, tail = rows - nfull * chunk;
  const int nch = int(nfull + (tail > 0 ? 1 : 0));
  if (nch < 1 || int64_t(nch) * M * N > net->parts_n || nfull > 65535) return STFD_EINVAL;
  int rc;
  if (nfull > 0)
    if ((rc = gemm(s, int(nfull), M, N, int(chunk), A, 1, M, chunk * M, B, N, 1, chunk * N, net->parts, N, 1,
                   int64_t(M) * N, nullptr, 1.0f, 0.0f)))
      return rc;
  if (tail > 0) {
    const int64_t r0 = nfull * chunk;
    if ((rc = gemm(s, 1, M, N, int(tail), A + r0 * M, 1, M, 0, B + r0 * N, N, 1, 0,
                   net->parts + nfull * int64_t(M) * N, N, 1, 0, nullptr, 1.0f, 0.0f)))
      return rc;
  }
  hipLaunchKernelGGL(sum_parts_kernel, dim3(grid_for(int64_t(M) * N)), dim3(256), 0, s, (const float*)net->parts, nch,
                     int64_t(M) * N, C, 0.0f);
  FNO_HIP(hipGetLastError());
  return STFD_OK;
}

int colsum(stfd_fno* net, hipStream_t s, const float* X, int64_t rows, int ncol, float* out) {
  const int64_t chunk = 1024;
  const int nch = int((rows + chunk - 1) / chunk);
  if (int64_t(nch) * ncol > net->parts_n) return STFD_EINVAL;
  hipLaunchKernelGGL(colsum_part_kernel, dim3(unsigned((ncol + 63) / 64), unsigned(nch)), dim3(256), 0, s, X, rows,
                     ncol, chunk, net->parts);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(grid_for(ncol)), dim3(256), 0, s, (const float*)net->parts, nch,
                     int64_t(ncol), out, 0.0f);
  FNO_HIP(hipGetLastError());
  return STFD_OK;
}

// SplitMix64 (Steele, Lea, Flood 2014) -> uniform [0, 1)
struct SplitMix {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return double(next() >> 11) * (1.0 / 9007199254740992.0); }
};

template <typename T>
int alloc(stfd_fno* net, T** p, size_t n) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T));
  if (e != hipSuccess) {
    g_hip_err = int(e);
    return STFD_ENOMEM;
  }
  net->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return STFD_OK;
}

}  // namespace

int stfd_fno_create(const stfd_fno_desc* desc, stfd_fno** out) {
  if (!desc || !out) return STFD_EINVAL;
  *out = nullptr;
  const stfd_fno_desc& d = *desc;
  if (d.H < 2 || d.W < 2 || d.c_in < 1 || d.width < 1 || d.layers < 1 || d.proj < 1 || d.c_out < 1 ||
      d.max_batch < 1 || d.modes1 < 1 || d.modes1 > d.W / 2 + 1 || d.modes2 < 2 || d.modes2 % 2 || d.modes2 > d.H)
    return STFD_EINVAL;
  stfd_fno* net = new (std::nothrow) stfd_fno;
  if (!net) return STFD_ENOMEM;
  net->d = d;
  const int C = d.width, M1 = d.modes1, M2 = d.modes2, L = d.layers, H = d.H, W = d.W;
  // parameter layout
  int64_t o = 0;
  net->oWp = o; o += int64_t(d.c_in) * C;
  net->obp = o; o += C;
  for (int l = 0; l < L; ++l) {
    net->oW.push_back(o); o += int64_t(C) * C;
    net->ob.push_back(o); o += C;
    net->oRr.push_back(o); o += int64_t(M2) * M1 * C * C;
    net->oRi.push_back(o); o += int64_t(M2) * M1 * C * C;
  }
  net->oQ1 = o; o += int64_t(C) * d.proj;
  net->oq1 = o; o += d.proj;
  net->oQ2 = o; o += int64_t(d.proj) * d.c_out;
  net->oq2 = o; o += d.c_out;
  net->nparams = o;
  std::vector<float> P(size_t(o), 0.0f);
  SplitMix rng{d.seed};
  auto fill = [&](int64_t off, int64_t n, double scale, bool symmetric) {
    for (int64_t i = 0; i < n; ++i) {
      const double u = rng.uniform();
      P[size_t(off + i)] = float(symmetric ? scale * (2.0 * u - 1.0) : scale * u);
    }
  };
  fill(net->oWp, int64_t(d.c_in) * C, 1.0 / std::sqrt(double(d.c_in)), true);
  for (int l = 0; l < L; ++l) {
    fill(net->oW[size_t(l)], int64_t(C) * C, 1.0 / std::sqrt(double(C)), true);
    fill(net->oRr[size_t(l)], int64_t(M2) * M1 * C * C, 1.0 / (double(C) * C), false);
    fill(net->oRi[size_t(l)], int64_t(M2) * M1 * C * C, 1.0 / (double(C) * C), false);
  }
  fill(net->oQ1, int64_t(C) * d.proj, 1.0 / std::sqrt(double(C)), true);
  fill(net->oQ2, int64_t(d.proj) * d.c_out, 1.0 / std::sqrt(double(d.proj)), true);
  // DFT matrices
  const double tp = 2.0 * M_PI;
  std::vector<float> D1(size_t(2 * M1) * W), D2(size_t(2 * M2) * 2 * H), E2(size_t(2 * H) * 2 * M2),
      E1(size_t(W) * 2 * M1);
  for (int k1 = 0; k1 < M1; ++k1)
    for (int i1 = 0; i1 < W; ++i1) {
      const double ang = tp * double((int64_t(k1) * i1) % W) / W;
      D1[size_t(k1) * W + i1] = float(std::cos(ang));
      D1[size_t(M1 + k1) * W + i1] = float(-std::sin(ang));
      const double wk = (k1 == 0 ? 1.0 : 2.0) / (double(H) * W);
      E1[size_t(i1) * 2 * M1 + k1] = float(wk * std::cos(ang));
      E1[size_t(i1) * 2 * M1 + M1 + k1] = float(-wk * std::sin(ang));
    }
  for (int j = 0; j < M2; ++j) {
    const int k2 = j < M2 / 2 ? j : j - M2;
    for (int i2 = 0; i2 < H; ++i2) {
      const int64_t kk = ((int64_t(k2) * i2) % H + H) % H;
      const double ang = tp * double(kk) / H;
      const double c = std::cos(ang), sn = std::sin(ang);
      // forward: X = sum exp(-i ang) Y: Xr = c Yr + s Yi, Xi = -s Yr + c Yi
      D2[size_t(2 * j) * 2 * H + 2 * i2] = float(c);
      D2[size_t(2 * j) * 2 * H + 2 * i2 + 1] = float(sn);
      D2[size_t(2 * j + 1) * 2 * H + 2 * i2] = float(-sn);
      D2[size_t(2 * j + 1) * 2 * H + 2 * i2 + 1] = float(c);
      // inverse: Z = sum exp(+i ang) X: Zr = c Xr - s Xi, Zi = s Xr + c Xi
      E2[size_t(2 * i2) * 2 * M2 + 2 * j] = float(c);
      E2[size_t(2 * i2) * 2 * M2 + 2 * j + 1] = float(-sn);
      E2[size_t(2 * i2 + 1) * 2 * M2 + 2 * j] = float(sn);
      E2[size_t(2 * i2 + 1) * 2 * M2 + 2 * j + 1] = float(c);
    }
  }
  const int64_t B = d.max_batch, HW = int64_t(H) * W;
  const int64_t nact = B * HW * C, nspec = B * 2 * M2 * M1 * C, nf1 = B * H * 2 * M1 * C;
  int rc = STFD_OK;
  auto A = [&](float** p, int64_t n) {
    if (rc == STFD_OK) rc = alloc(net, p, size_t(n));
  };
  A(&net->params, o);
  A(&net->grads, o);
  A(&net->adam_m, o);
  A(&net->adam_v, o);
  A(&net->D1, int64_t(D1.size()));
  A(&net->D2, int64_t(D2.size()));
  A(&net->E2, int64_t(E2.size()));
  A(&net->E1, int64_t(E1.size()));
  A(&net->x, B * HW * d.c_in);
  net->a.resize(size_t(L + 1), nullptr);
  net->z.resize(size_t(L), nullptr);
  net->Xs.resize(size_t(L), nullptr);
  for (int l = 0; l <= L; ++l)
    if (l < L) A(&net->a[size_t(l)], nact);
  for (int l = 0; l < L; ++l) {
    A(&net->z[size_t(l)], nact);
    A(&net->Xs[size_t(l)], nspec);
  }
  net->a[size_t(L)] = nullptr;  // a_L aliases z_{L-1}
  A(&net->F1, nf1);
  A(&net->Ybuf, nspec);
  A(&net->T2, nf1);
  A(&net->p1, B * HW * d.proj);
  A(&net->g1, B * HW * d.proj);
  const int64_t wide = std::max<int64_t>(std::max(C, d.proj), d.c_in);
  A(&net->da, B * HW * wide);
  A(&net->dz, B * HW * wide);
  A(&net->dp, B * HW * d.proj);
  A(&net->dX, std::max(nspec, nf1));
  const int64_t mx = std::max<int64_t>(std::max<int64_t>(C, d.proj), std::max<int64_t>(d.c_in, d.c_out));
  net->parts_n = ((B * HW + 1023) / 1024 + 1) * mx * mx + 4096;
  A(&net->parts, net->parts_n);
  A(&net->scal, B + 1);
  if (rc) {
    stfd_fno_destroy(net);
    return rc;
  }
  net->a[size_t(L)] = net->z[size_t(L - 1)];
  hipError_t e = hipMemcpy(net->params, P.data(), P.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(net->D1, D1.data(), D1.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(net->D2, D2.data(), D2.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(net->E2, E2.data(), E2.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(net->E1, E1.data(), E1.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(net->grads, 0, size_t(o) * sizeof(float));
  if (e == hipSuccess) e = hipMemset(net->adam_m, 0, size_t(o) * sizeof(float));
  if (e == hipSuccess) e = hipMemset(net->adam_v, 0, size_t(o) * sizeof(float));
  if (e != hipSuccess) {
    g_hip_err = int(e);
    stfd_fno_destroy(net);
    return STFD_EHIP;
  }
  *out = net;
  return STFD_OK;
}

void stfd_fno_destroy(stfd_fno* net) {
  if (!net) return;
  for (void* p : net->allocs) (void)hipFree(p);
  delete net;
}

int stfd_fno_num_params(const stfd_fno* net, int64_t* n) {
  if (!net || !n) return STFD_EINVAL;
  *n = net->nparams;
  return STFD_OK;
}

int stfd_fno_get_params(const stfd_fno* net, float* host) {
  if (!net || !host) return STFD_EINVAL;
  FNO_HIP(hipMemcpy(host, net->params, size_t(net->nparams) * sizeof(float), hipMemcpyDeviceToHost));
  return STFD_OK;
}

int stfd_fno_set_params(stfd_fno* net, const float* host) {
  if (!net || !host) return STFD_EINVAL;
  FNO_HIP(hipMemcpy(net->params, host, size_t(net->nparams) * sizeof(float), hipMemcpyHostToDevice));
  return STFD_OK;
}

int stfd_fno_get_grads(const stfd_fno* net, float* host) {
  if (!net || !host) return STFD_EINVAL;
  FNO_HIP(hipMemcpy(host, net->grads, size_t(net->nparams) * sizeof(float), hipMemcpyDeviceToHost));
  return STFD_OK;
}

int stfd_fno_forward(stfd_fno* net, const float* x_dev, float* y_dev, int batch, void* stream) {
  if (!net || !x_dev || !y_dev || batch < 1 || batch > net->d.max_batch) return STFD_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const stfd_fno_desc& d = net->d;
  const int C = d.width, M1 = d.modes1, M2 = d.modes2, L = d.layers, H = d.H, W = d.W;
  const int64_t HW = int64_t(H) * W, rows = int64_t(batch) * HW;
  const float* P = net->params;
  int rc;
  FNO_HIP(hipMemcpyAsync(net->x, x_dev, size_t(rows) * d.c_in * sizeof(float), hipMemcpyDeviceToDevice, s));
  // lift
  if ((rc = gemm(s, 1, int(rows), C, d.c_in, net->x, d.c_in, 1, 0, P + net->oWp, C, 1, 0, net->a[0], C, 1, 0,
                 P + net->obp, 1.0f, 0.0f)))
    return rc;
  for (int l = 0; l < L; ++l) {
    const float* al = net->a[size_t(l)];
    float* zl = net->z[size_t(l)];
    float* Xl = net->Xs[size_t(l)];
    // F1 = DFT along i_1, per (b, i_2): [2 M1 x W] [W x C]
    if ((rc = gemm(s, batch * H, 2 * M1, C, W, net->D1, W, 1, 0, al, C, 1, int64_t(W) * C, net->F1, C, 1,
                   int64_t(2 * M1) * C, nullptr, 1.0f, 0.0f)))
      return rc;
    // X = DFT along i_2, per b: [2 M2 x 2 H] [2 H x M1 C]
    if ((rc = gemm(s, batch, 2 * M2, M1 * C, 2 * H, net->D2, 2 * H, 1, 0, net->F1, int64_t(M1) * C, 1,
                   int64_t(H) * 2 * M1 * C, Xl, int64_t(M1) * C, 1, int64_t(2 * M2) * M1 * C, nullptr, 1.0f, 0.0f)))
      return rc;
    hipLaunchKernelGGL(mix_fwd_kernel, dim3(grid_for(int64_t(batch) * M2 * M1 * C)), dim3(256), 0, s,
                       (const float*)Xl, P + net->oRr[size_t(l)], P + net->oRi[size_t(l)], net->Ybuf, batch, M1, M2, C);
    FNO_HIP(hipGetLastError());
    // T2 = inverse along i_2: [2 H x 2 M2] [2 M2 x M1 C]
    if ((rc = gemm(s, batch, 2 * H, M1 * C, 2 * M2, net->E2, 2 * M2, 1, 0, net->Ybuf, int64_t(M1) * C, 1,
                   int64_t(2 * M2) * M1 * C, net->T2, int64_t(M1) * C, 1, int64_t(H) * 2 * M1 * C, nullptr, 1.0f,
                   0.0f)))
      return rc;
    // z = inverse along i_1 (real part): [W x 2 M1] [2 M1 x C], then z += a W_l + b_l
    if ((rc = gemm(s, batch * H, W, C, 2 * M1, net->E1, 2 * M1, 1, 0, net->T2, C, 1, int64_t(2 * M1) * C, zl, C, 1,
                   int64_t(W) * C, nullptr, 1.0f, 0.0f)))
      return rc;
    if ((rc = gemm(s, 1, int(rows), C, C, al, C, 1, 0, P + net->oW[size_t(l)], C, 1, 0, zl, C, 1, 0,
                   P + net->ob[size_t(l)], 1.0f, 1.0f)))
      return rc;
    if (l < L - 1) {
      hipLaunchKernelGGL(gelu_kernel, dim3(grid_for(rows * C)), dim3(256), 0, s, (const float*)zl, net->a[size_t(l + 1)],
                         rows * C);
      FNO_HIP(hipGetLastError());
    }
  }
  // projection
  if ((rc = gemm(s, 1, int(rows), d.proj, C, net->a[size_t(L)], C, 1, 0, P + net->oQ1, d.proj, 1, 0, net->p1, d.proj,
                 1, 0, P + net->oq1, 1.0f, 0.0f)))
    return rc;
  hipLaunchKernelGGL(gelu_kernel, dim3(grid_for(rows * d.proj)), dim3(256), 0, s, (const float*)net->p1, net->g1,
                     rows * d.proj);
  FNO_HIP(hipGetLastError());
  if ((rc = gemm(s, 1, int(rows), d.c_out, d.proj, net->g1, d.proj, 1, 0, P + net->oQ2, d.c_out, 1, 0, y_dev, d.c_out,
                 1, 0, P + net->oq2, 1.0f, 0.0f)))
    return rc;
  net->last_batch = batch;
  return STFD_OK;
}

int stfd_fno_backward(stfd_fno* net, const float* dy_dev, float* dx_dev, int batch, void* stream) {
  if (!net || !dy_dev || batch < 1 || batch != net->last_batch) return STFD_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const stfd_fno_desc& d = net->d;
  const int C = d.width, M1 = d.modes1, M2 = d.modes2, L = d.layers, H = d.H, W = d.W;
  const int64_t HW = int64_t(H) * W, rows = int64_t(batch) * HW;
  const float* P = net->params;
  float* G = net->grads;
  int rc;
  // y = g1 Q2 + q2
  if ((rc = wgrad(net, s, rows, d.proj, d.c_out, net->g1, dy_dev, G + net->oQ2))) return rc;
  if ((rc = colsum(net, s, dy_dev, rows, d.c_out, G + net->oq2))) return rc;
  // dg1 = dy Q2^T -> dp = dg1 * GELU'(p1)
  if ((rc = gemm(s, 1, int(rows), d.proj, d.c_out, dy_dev, d.c_out, 1, 0, P + net->oQ2, 1, d.c_out, 0, net->dp,
                 d.proj, 1, 0, nullptr, 1.0f, 0.0f)))
    return rc;
  hipLaunchKernelGGL(gelu_bwd_kernel, dim3(grid_for(rows * d.proj)), dim3(256), 0, s, (const float*)net->p1,
                     (const float*)net->dp, net->dp, rows * d.proj);
  FNO_HIP(hipGetLastError());
  // p1 = a_L Q1 + q1
  if ((rc = wgrad(net, s, rows, C, d.proj, net->a[size_t(L)], net->dp, G + net->oQ1))) return rc;
  if ((rc = colsum(net, s, net->dp, rows, d.proj, G + net->oq1))) return rc;
  // dz_{L-1} = da_L = dp Q1^T
  if ((rc = gemm(s, 1, int(rows), C, d.proj, net->dp, d.proj, 1, 0, P + net->oQ1, 1, d.proj, 0, net->dz, C, 1, 0,
                 nullptr, 1.0f, 0.0f)))
    return rc;
  for (int l = L - 1; l >= 0; --l) {
    const float* al = net->a[size_t(l)];
    // dz holds dz_l.  Parameters of the pointwise part.
    if ((rc = wgrad(net, s, rows, C, C, al, net->dz, G + net->oW[size_t(l)]))) return rc;
    if ((rc = colsum(net, s, net->dz, rows, C, G + net->ob[size_t(l)]))) return rc;
    // da = dz W_l^T
    if ((rc = gemm(s, 1, int(rows), C, C, net->dz, C, 1, 0, P + net->oW[size_t(l)], 1, C, 0, net->da, C, 1, 0,
                   nullptr, 1.0f, 0.0f)))
      return rc;
    // spectral adjoint: dT2 = E1^T dz (per (b, i_2)): [2 M1 x W] [W x C]
    if ((rc = gemm(s, batch * H, 2 * M1, C, W, net->E1, 1, 2 * M1, 0, net->dz, C, 1, int64_t(W) * C, net->T2, C, 1,
                   int64_t(2 * M1) * C, nullptr, 1.0f, 0.0f)))
      return rc;
    // dY = E2^T dT2 (per b): [2 M2 x 2 H] [2 H x M1 C]
    if ((rc = gemm(s, batch, 2 * M2, M1 * C, 2 * H, net->E2, 1, 2 * M2, 0, net->T2, int64_t(M1) * C, 1,
                   int64_t(H) * 2 * M1 * C, net->Ybuf, int64_t(M1) * C, 1, int64_t(2 * M2) * M1 * C, nullptr, 1.0f,
                   0.0f)))
      return rc;
    hipLaunchKernelGGL(mix_bwd_w_kernel, dim3(grid_for(int64_t(M2) * M1 * C * C)), dim3(256), 0, s,
                       (const float*)net->Xs[size_t(l)], (const float*)net->Ybuf, G + net->oRr[size_t(l)],
                       G + net->oRi[size_t(l)], batch, M1, M2, C);
    hipLaunchKernelGGL(mix_bwd_in_kernel, dim3(grid_for(int64_t(batch) * M2 * M1 * C)), dim3(256), 0, s,
                       (const float*)net->Ybuf, P + net->oRr[size_t(l)], P + net->oRi[size_t(l)], net->dX, batch, M1,
                       M2, C);
    FNO_HIP(hipGetLastError());
    // dF1 = D2^T dX (per b): [2 H x 2 M2] [2 M2 x M1 C]
    if ((rc = gemm(s, batch, 2 * H, M1 * C, 2 * M2, net->D2, 1, 2 * H, 0, net->dX, int64_t(M1) * C, 1,
                   int64_t(2 * M2) * M1 * C, net->F1, int64_t(M1) * C, 1, int64_t(H) * 2 * M1 * C, nullptr, 1.0f,
                   0.0f)))
      return rc;
    // da += D1^T dF1 (per (b, i_2)): [W x 2 M1] [2 M1 x C]
    if ((rc = gemm(s, batch * H, W, C, 2 * M1, net->D1, 1, W, 0, net->F1, C, 1, int64_t(2 * M1) * C, net->da, C, 1,
                   int64_t(W) * C, nullptr, 1.0f, 1.0f)))
      return rc;
    if (l > 0) {
      hipLaunchKernelGGL(gelu_bwd_kernel, dim3(grid_for(rows * C)), dim3(256), 0, s, (const float*)net->z[size_t(l - 1)],
                         (const float*)net->da, net->dz, rows * C);
      FNO_HIP(hipGetLastError());
    }
  }
  // lift: a_0 = x Wp + bp, da holds da_0
  if ((rc = wgrad(net, s, rows, d.c_in, C, net->x, net->da, G + net->oWp))) return rc;
  if ((rc = colsum(net, s, net->da, rows, C, G + net->obp))) return rc;
  if (dx_dev)
    if ((rc = gemm(s, 1, int(rows), d.c_in, C, net->da, C, 1, 0, P + net->oWp, 1, C, 0, dx_dev, d.c_in, 1, 0, nullptr,
                   1.0f, 0.0f)))
      return rc;
  return STFD_OK;
}

int stfd_fno_rel_l2(const float* y_dev, const float* t_dev, int64_t n, int batch, float* dy_dev, float* loss,
                    void* stream) {
  if (!y_dev || !t_dev || n < 1 || batch < 1 || batch > 65535) return STFD_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nparts = 64;
  float* scratch = nullptr;
  FNO_HIP(hipMalloc(reinterpret_cast<void**>(&scratch), (size_t(batch) * nparts * 2 + batch + 1) * sizeof(float)));
  float* scal = scratch + size_t(batch) * nparts * 2;
  hipLaunchKernelGGL(rel_l2_part_kernel, dim3(nparts, unsigned(batch)), dim3(256), 0, s, y_dev, t_dev, n, scratch);
  hipLaunchKernelGGL(rel_l2_final_kernel, dim3(1), dim3(64), 0, s, (const float*)scratch, nparts, batch, scal);
  if (dy_dev)
    hipLaunchKernelGGL(rel_l2_grad_kernel, dim3(unsigned(grid_for(n) > 1024 ? 1024 : grid_for(n)), unsigned(batch)),
                       dim3(256), 0, s, y_dev, t_dev, (const float*)scal, n, dy_dev);
  hipError_t e = hipGetLastError();
  float lv = 0.0f;
  if (e == hipSuccess) e = hipMemcpyAsync(&lv, scal, sizeof(float), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(scratch);
  if (e != hipSuccess) {
    g_hip_err = int(e);
    return STFD_EHIP;
  }
  if (loss) *loss = lv;
  return STFD_OK;
}

int stfd_fno_adam_step(stfd_fno* net, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!net || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return STFD_EINVAL;
  net->step += 1;
  const float bc1 = 1.0f - std::pow(beta1, float(net->step));
  const float bc2 = 1.0f - std::pow(beta2, float(net->step));
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(net->nparams)), dim3(256), 0, static_cast<hipStream_t>(stream),
                     net->params, (const float*)net->grads, net->adam_m, net->adam_v, net->nparams, lr, beta1, beta2,
                     eps, bc1, bc2);
  FNO_HIP(hipGetLastError());
  return STFD_OK;
}

int stfd_fno_to_f64(const float* y_dev, double* x_dev, int64_t n, void* stream) {
  if (!y_dev || !x_dev || n < 0) return STFD_EINVAL;
  if (n == 0) return STFD_OK;
  hipLaunchKernelGGL(to_f64_kernel, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), y_dev, x_dev,
                     n);
  FNO_HIP(hipGetLastError());
  return STFD_OK;
}

int stfd_fno_diff_f64(const float* y_dev, const float* t_dev, double* e_dev, int64_t n, void* stream) {
  if (!y_dev || !e_dev || n < 0) return STFD_EINVAL;
  if (n == 0) return STFD_OK;
  hipLaunchKernelGGL(diff_f64_kernel, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), y_dev, t_dev,
                     e_dev, n);
  FNO_HIP(hipGetLastError());
  return STFD_OK;
}

int stfd_fno_energy_loss(const double* e_dev, const double* Ae_dev, const double* t_energy_dev, int64_t n, int batch,
                         float* dy_dev, double* energy_host, float* loss, void* stream) {
  if (!e_dev || !Ae_dev || n < 1 || batch < 1 || batch > 65535) return STFD_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nparts = 64;
  double* scratch = nullptr;
  FNO_HIP(hipMalloc(reinterpret_cast<void**>(&scratch), (size_t(batch) * nparts + 2 + 2 * size_t(batch)) * sizeof(double)));
  double* scal = scratch + size_t(batch) * nparts;
  hipLaunchKernelGGL(energy_part_kernel, dim3(nparts, unsigned(batch)), dim3(256), 0, s, e_dev, Ae_dev, n, scratch);
  hipLaunchKernelGGL(energy_final_kernel, dim3(1), dim3(64), 0, s, (const double*)scratch, nparts, batch, t_energy_dev,
                     scal);
  if (dy_dev)
    hipLaunchKernelGGL(energy_grad_kernel, dim3(unsigned(std::min(grid_for(n), 1024)), unsigned(batch)), dim3(256), 0,
                       s, Ae_dev, (const double*)scal, n, dy_dev);
  hipError_t e = hipGetLastError();
  std::vector<double> host(2 + 2 * size_t(batch));
  if (e == hipSuccess) e = hipMemcpyAsync(host.data(), scal, host.size() * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(scratch);
  if (e != hipSuccess) {
    g_hip_err = int(e);
    return STFD_EHIP;
  }
  if (loss) *loss = float(host[0]);
  if (energy_host)
    for (int b = 0; b < batch; ++b) energy_host[b] = host[2 + size_t(batch) + b];
  return STFD_OK;
}
