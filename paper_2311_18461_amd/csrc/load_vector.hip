// Lifting and load vector on the device (Sections 2.2 and 4.3).
//
// With u = u_free + u_bar (u_bar the lifting of the initial and Dirichlet
// data), the free coefficients solve A u_free = f_bar with
//   f_bar_I = integral over (0,T) x Omega of (f - S_V u_bar) conj(S_V B_I),
// S_V = i d_t - nu Lap + V.  The B-splines are real, so
//   conj(S_V B_I) = -i b_t' phi - nu b_t Lap phi + V b_t phi.
// Everything is sum-factorised on the tensor Gauss grid:
//   evaluation  A0 = (B_1^T (x) ... (x) B_d^T) G,  A2 = sum_l (... B_l''^T ...) G  (space first)
//               R  = f - i B_t'^T A0 + B_t^T (nu A2 - V A0)                      (R = f - S_V u_bar)
//   load        X0 = B_t^w R,  X1 = B_t'^w R                                      (time first)
//               f_bar = (B_1^w (x) ... (x) B_d^w)(-i X1 + V X0) - nu sum_l (... B_l''^w ...) X0
// where ^w marks the weighted free-row matrices.  V does not depend on t, so it
// commutes with every time contraction.
//
// Lifting u_bar: the coefficients of the B-splines that do not vanish on Gamma
// (initial face and lateral faces) minimise sum_F ||u_bar - data_F||^2_{L2(F)}.
// On face F only the functions with index normal_index along the normal axis
// are non-zero (b_0(0) = 1 in time, phi_0(0) = phi_{m-1}(1) = 1 in space), so
// the normal equations are (sum_F P_F^T M_F P_F) g = sum_F P_F^T b_F with M_F the
// Kronecker product of the full 1D mass matrices tangent to F.  They are solved
// by CG preconditioned with the overlapping additive Schwarz operator
// sum_F P_F^T M_F^{-1} P_F (dense 1D inverses applied axis by axis).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "load_vector.h"

namespace stfd {

constexpr int kContractBatch = 8;
constexpr int kLiftBatch = 24;

// out[o][i][r] = alpha * sum_{k in [lo_i, hi_i)} M[i * ld + k] in[o][k][r]  (+ out if accumulate)
__global__ void __launch_bounds__(256) axis_contract_kernel(const double2* __restrict__ in, double2* __restrict__ out,
                                                            const double* __restrict__ M, const int* __restrict__ lo,
                                                            const int* __restrict__ hi, int ld, int n_out, int n_in,
                                                            int64_t inner, int64_t total, double ar, double ai,
                                                            int accumulate) {
  for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total; g += int64_t(gridDim.x) * blockDim.x) {
    const int64_t r = g % inner;
    const int64_t t = g / inner;
    const int i = int(t % n_out);
    const int64_t o = t / n_out;
    const double2* src = in + o * n_in * inner + r;
    const double* row = M + int64_t(i) * ld;
    double sr = 0.0, si = 0.0;
    // the band in batches whose loads are all issued before any is used (addresses clamped
    // into the band, coefficients of the clamped slots zero)
    const int k0 = lo[i], k1 = hi[i];
    for (int kb = k0; kb < k1; kb += kContractBatch) {
      double c[kContractBatch];
      double2 v[kContractBatch];
#pragma unroll
      for (int u = 0; u < kContractBatch; ++u) {
        const int k = min(kb + u, k1 - 1);
        c[u] = kb + u < k1 ? row[k] : 0.0;
        v[u] = src[int64_t(k) * inner];
      }
#pragma unroll
      for (int u = 0; u < kContractBatch; ++u) {
        sr = fma(c[u], v[u].x, sr);
        si = fma(c[u], v[u].y, si);
      }
    }
    double2 res;
    res.x = ar * sr - ai * si;
    res.y = ar * si + ai * sr;
    if (accumulate) {
      const double2 prev = out[g];
      res.x += prev.x;
      res.y += prev.y;
    }
    out[g] = res;
  }
}

// Time axis (the fastest one) of the load vector, one block per spatial grid point o, the point's
// time line staged in LDS:
//   time_expand: R[o][q] = f[o][q] - i sum_k E1[q][k] A[o][k] + sum_k E0[q][k] C[o][k]
//                (f == nullptr: 0), E0 / E1 the time basis and its derivative at the Gauss points;
//   (both matrices as transposed bands band[u][row] = M[row][lo_row + u]);
//   time_load:   X0[o][i] = sum_q L0[i][q] R[o][q],  X1[o][i] = sum_q L1[i][q] R[o][q],
//                Y[o][i] = J[o] (-i X1 + V[o] X0)  (V == nullptr drops the term, J == nullptr: 1).
// R at time Gauss point q of one spatial point, from the point's A and C (tl[0..m), tl[m..2m)).
__device__ __forceinline__ double2 time_expand_at(const double2* tl, int m, int q, int Q, const double* E0b,
                                                  const double* E1b, const int* lo, int ew) {
  double ar = 0.0, ai = 0.0, cr = 0.0, ci = 0.0;
  const int k0 = lo[q];
  for (int u = 0; u < ew; ++u) {
    const int k = min(k0 + u, m - 1);  // slots past the row's band carry zero weights
    const double e0 = E0b[int64_t(u) * Q + q], e1 = E1b[int64_t(u) * Q + q];
    const double2 a = tl[k], c = tl[m + k];
    ar = fma(e1, a.x, ar);
    ai = fma(e1, a.y, ai);
    cr = fma(e0, c.x, cr);
    ci = fma(e0, c.y, ci);
  }
  return make_double2(ai + cr, ci - ar);  // -i (ar + i ai) + (cr + i ci)
}
// X0 and Y at free time row i of one spatial point, from the point's R (tl[0..Q)).
__device__ __forceinline__ void time_load_at(const double2* tl, int Q, int i, int n, const double* L0b,
                                             const double* L1b, const int* lo, int lw, double v, double jac,
                                             double2& x0, double2& y) {
  double x0r = 0.0, x0i = 0.0, x1r = 0.0, x1i = 0.0;
  const int q0 = lo[i];
  for (int u = 0; u < lw; ++u) {
    const int q = min(q0 + u, Q - 1);  // slots past the row's band carry zero weights
    const double l0 = L0b[int64_t(u) * n + i], l1 = L1b[int64_t(u) * n + i];
    const double2 r = tl[q];
    x0r = fma(l0, r.x, x0r);
    x0i = fma(l0, r.y, x0i);
    x1r = fma(l1, r.x, x1r);
    x1i = fma(l1, r.y, x1i);
  }
  x0 = make_double2(x0r, x0i);
  y = make_double2(jac * (x1i + v * x0r), jac * (v * x0i - x1r));
}

__global__ void __launch_bounds__(256) time_expand_kernel(const double2* __restrict__ A, const double2* __restrict__ C,
                                                          const double2* __restrict__ f, double2* __restrict__ R,
                                                          const double* __restrict__ E0b, const double* __restrict__ E1b,
                                                          const int* __restrict__ lo, int ew, int m, int Q) {
  extern __shared__ double2 tl[];  // [2][m]: A and C of this point
  const int64_t o = blockIdx.x;
  for (int k = threadIdx.x; k < m; k += blockDim.x) {
    tl[k] = A[o * m + k];
    tl[m + k] = C[o * m + k];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < Q; q += blockDim.x) {
    double2 res = time_expand_at(tl, m, q, Q, E0b, E1b, lo, ew);
    if (f) {
      const double2 fv = f[o * Q + q];
      res.x += fv.x;
      res.y += fv.y;
    }
    R[o * Q + q] = res;
  }
}

__global__ void __launch_bounds__(256) time_load_kernel(const double2* __restrict__ R, double2* __restrict__ X0,
                                                        double2* __restrict__ Y, const double* __restrict__ L0b,
                                                        const double* __restrict__ L1b, const int* __restrict__ lo,
                                                        int lw, int Q, int n, const double* __restrict__ V,
                                                        const double* __restrict__ J) {
  extern __shared__ double2 tl[];  // [Q]: R of this point
  const int64_t o = blockIdx.x;
  for (int q = threadIdx.x; q < Q; q += blockDim.x) tl[q] = R[o * Q + q];
  __syncthreads();
  const double v = V ? V[o] : 0.0, jac = J ? J[o] : 1.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    time_load_at(tl, Q, i, n, L0b, L1b, lo, lw, v, jac, X0[o * n + i], Y[o * n + i]);
}

// time_expand and time_load in one launch where a point's A, C and R fit in LDS: R stays in LDS
// instead of a round trip of the whole space-time Gauss grid through memory (268 MB at 64^3); the
// same arithmetic in the same order, so the same results.
constexpr size_t kTimeRhsMaxLds = 64 * 1024;
__global__ void __launch_bounds__(256) time_rhs_kernel(const double2* __restrict__ A, const double2* __restrict__ C,
                                                       const double2* __restrict__ f, const double* __restrict__ E0b,
                                                       const double* __restrict__ E1b, const int* __restrict__ elo,
                                                       int ew, int m, int Q, double2* __restrict__ X0,
                                                       double2* __restrict__ Y, const double* __restrict__ L0b,
                                                       const double* __restrict__ L1b, const int* __restrict__ llo,
                                                       int lw, int n, const double* __restrict__ V,
                                                       const double* __restrict__ J) {
  extern __shared__ double2 tl[];  // [2][m]: A and C of this point, then [Q]: its R
  double2* Rs = tl + 2 * m;
  const int64_t o = blockIdx.x;
  for (int k = threadIdx.x; k < m; k += blockDim.x) {
    tl[k] = A[o * m + k];
    tl[m + k] = C[o * m + k];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < Q; q += blockDim.x) {
    double2 res = time_expand_at(tl, m, q, Q, E0b, E1b, elo, ew);
    if (f) {
      const double2 fv = f[o * Q + q];
      res.x += fv.x;
      res.y += fv.y;
    }
    Rs[q] = res;
  }
  __syncthreads();
  const double v = V ? V[o] : 0.0, jac = J ? J[o] : 1.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    time_load_at(Rs, Q, i, n, L0b, L1b, llo, lw, v, jac, X0[o * n + i], Y[o * n + i]);
}

// out[x][t] = J[x] (alpha A[x][t] + beta V[x] B[x][t])  (t fastest, n_time entries per x;
// V == nullptr drops the second term, J == nullptr means J = 1)
__global__ void __launch_bounds__(256) combine_v_kernel(const double2* __restrict__ A, const double2* __restrict__ B,
                                                        const double* __restrict__ V, const double* __restrict__ J,
                                                        double2* __restrict__ out, int64_t n_time, int64_t total,
                                                        double ar, double ai, double beta) {
  for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total; g += int64_t(gridDim.x) * blockDim.x) {
    const double2 a = A[g];
    double2 res;
    res.x = ar * a.x - ai * a.y;
    res.y = ar * a.y + ai * a.x;
    if (V) {
      const double s = beta * V[g / n_time];
      const double2 b = B[g];
      res.x = fma(s, b.x, res.x);
      res.y = fma(s, b.y, res.y);
    }
    if (J) {
      const double j = J[g / n_time];
      res.x *= j;
      res.y *= j;
    }
    out[g] = res;
  }
}

// out[x][t] += c[x] A[x][t]
__global__ void __launch_bounds__(256) scale_add_kernel(const double2* __restrict__ A, const double* __restrict__ c,
                                                        double2* __restrict__ out, int64_t n_time, int64_t total,
                                                        double scale, int accumulate) {
  for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total; g += int64_t(gridDim.x) * blockDim.x) {
    const double f = scale * c[g / n_time];
    const double2 a = A[g];
    double2 res = make_double2(f * a.x, f * a.y);
    if (accumulate) {
      const double2 o = out[g];
      res.x += o.x;
      res.y += o.y;
    }
    out[g] = res;
  }
}

__global__ void __launch_bounds__(256) zero_kernel(double* __restrict__ x, int64_t n) {
  for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < n; g += int64_t(gridDim.x) * blockDim.x)
    x[g] = 0.0;
}

namespace {

int grid_for(int64_t total) { return int(std::min<int64_t>((total + 255) / 256, 8192)); }

// dynamic LDS beyond the default per-block limit (long time axes: the time-direction kernels stage
// one point's time line) is granted per kernel before the launch
int allow_lds(const void* fn, size_t bytes) {
  if (bytes <= 64 * 1024) return 0;
  return int(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)));
}

template <typename T>
int plan_upload(LoadPlan& plan, T** dst, const std::vector<T>& src) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, std::max<size_t>(src.size(), 1) * sizeof(T));
  if (e != hipSuccess) return int(e);
  plan.allocs.push_back(p);
  e = hipMemcpy(p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return int(e);
  *dst = static_cast<T*>(p);
  return 0;
}

// A tensor whose axes are (time, x_1, ..., x_d) with current extents dims[].
struct Shape {
  int na;
  int64_t dims[4];
};

// Contract axis a of `in` (extent dims[a]) into extent n_out with matrix M (n_out x ld).
int contract(const double* in, double* out, Shape& sh, int a, const double* M, const int* lo, const int* hi, int ld,
             int n_out, double ar, double ai, bool accumulate, hipStream_t s) {
  int64_t inner = 1;
  for (int b = 0; b < a; ++b) inner *= sh.dims[b];
  int64_t outer = 1;
  for (int b = a + 1; b < sh.na; ++b) outer *= sh.dims[b];
  const int n_in = int(sh.dims[a]);
  const int64_t total = outer * n_out * inner;
  sh.dims[a] = n_out;
  if (total == 0) return 0;
  hipLaunchKernelGGL(axis_contract_kernel, dim3(grid_for(total)), dim3(256), 0, s, (const double2*)in,
                     (double2*)out, M, lo, hi, ld, n_out, n_in, inner, total, ar, ai, accumulate ? 1 : 0);
  return int(hipGetLastError());
}

}  // namespace

// ---------------------------------------------------------------------------
// lifting kernels (fixed set of size n_fixed, faces packed in LiftFaces)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum64(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

struct LiftState {
  double bn, rz, alpha, beta, rn;
  int done;  // 0 running, 1 converged, 2 breakdown, 3 iteration limit
  int iters;
};

struct LiftArgs {
  LiftFaces fc;
  const int64_t* fixed;
  const int* fixed_idx;  // [n_fixed][4]
  const int* pos;
  int64_t n_fixed;
  const double* Mband[4];
  const double* Minv[4];
};

constexpr double kLiftTol2 = 1e-28;  // (relative residual 1e-14)^2

// Sum of one double over a 256-thread block (wave reductions, then LDS).
__device__ __forceinline__ double block_sum256(double v, double* lds) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) t = (lds[0] + lds[1]) + (lds[2] + lds[3]);
  __syncthreads();
  return t;
}

// Index along each axis of fixed unknown i (decoded on the host: one 16-byte load instead of 64-bit
// divisions per axis).
__device__ __forceinline__ void fixed_index(const LiftArgs& A, int64_t i, int* idx) {
  const int4 v = reinterpret_cast<const int4*>(A.fixed_idx)[i];
  idx[0] = v.x;
  idx[1] = v.y;
  idx[2] = v.z;
  idx[3] = v.w;
}

// y = (sum_F P_F^T M_F P_F) x on the fixed set, partials of Re <x, y> per block.  One wave per fixed
// unknown, lanes over the (flattened) tangent window of each face that contains it, so that a
// face costs one round of gathers and a wave reduction.
constexpr int kLiftMvWaves = 4;
__global__ void __launch_bounds__(64 * kLiftMvWaves) lift_matvec_kernel(LiftArgs A, const double2* __restrict__ x,
                                                                       double2* __restrict__ y,
                                                                       double* __restrict__ part,
                                                                       const LiftState* __restrict__ st) {
  __shared__ double red[kLiftMvWaves];
  if (st->done) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = int64_t(blockIdx.x) * kLiftMvWaves + wave;
  double acc_xy = 0.0;
  if (i < A.n_fixed) {
    // x[i] (for <x, y>) is loaded with the index: it does not wait for the gathers
    const double2 xv = x[i];
    const int64_t g = A.fixed[i];
    int idx[4];
    fixed_index(A, i, idx);
    double yr = 0.0, yi = 0.0;
    for (int f = 0; f < A.fc.count; ++f) {
      const LiftFace& F = A.fc.f[f];
      if (idx[F.normal_axis] != F.normal_index) continue;
      int lo[3] = {0, 0, 0}, len[3] = {1, 1, 1}, ax[3] = {0, 0, 0};
      int nwin = 1;
      for (int k = 0; k < F.n_tan; ++k) {
        ax[k] = F.tan_axis[k];
        const int pa = A.fc.p[ax[k]];
        lo[k] = max(0, idx[ax[k]] - pa);
        len[k] = min(A.fc.m[ax[k]] - 1, idx[ax[k]] + pa) - lo[k] + 1;
        nwin *= len[k];
      }
      for (int w0 = 0; w0 < nwin; w0 += 64) {
        const int wi = w0 + lane;
        if (wi < nwin) {
          int rest = wi;
          double c = 1.0;
          int64_t gu = g;
          for (int k = 0; k < F.n_tan; ++k) {
            const int j = lo[k] + rest % len[k];
            rest /= len[k];
            const int pa = A.fc.p[ax[k]];
            c *= A.Mband[ax[k]][idx[ax[k]] * (2 * pa + 1) + j - idx[ax[k]] + pa];
            gu += int64_t(j - idx[ax[k]]) * A.fc.stride[ax[k]];
          }
          const double2 v = x[A.pos[gu]];
          yr = fma(c, v.x, yr);
          yi = fma(c, v.y, yi);
        }
      }
    }
    yr = wave_sum64(yr);
    yi = wave_sum64(yi);
    if (lane == 0) {
      y[i] = make_double2(yr, yi);
      acc_xy = xv.x * yr + xv.y * yi;
    }
  }
  if (lane == 0) red[wave] = acc_xy;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kLiftMvWaves; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

// One axis of the face-wise inverse: out[F][loc] = sum_j Minv[ax][i_s][j] in_F(loc with i_s := j),
// in_F read from the fixed-set vector r (step 0) or from the packed buffer `in` (later steps).
// One thread per face entry and a dense row of the 1D inverse (m_l values) per entry: the launch
// holds a few hundred waves, so the row is read in batches of kLiftBatch loads (3 batches for
// m_l = 67 instead of 9), each batch one memory round trip (two at step 0: index, then value).
__global__ void __launch_bounds__(256) lift_prec_axis_kernel(LiftArgs A, int step, const double2* __restrict__ r,
                                                             const double2* __restrict__ in,
                                                             double2* __restrict__ out,
                                                             const LiftState* __restrict__ st) {
  if (st->done) return;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < A.fc.total; e += int64_t(gridDim.x) * blockDim.x) {
    int f = 0;
    while (f + 1 < A.fc.count && e >= A.fc.f[f + 1].offset) ++f;
    const LiftFace& F = A.fc.f[f];
    const int64_t loc = e - F.offset;
    int li[3] = {0, 0, 0};
    int64_t lstride[3] = {1, 1, 1};
    {
      // a face holds at most a few million entries (the setup size limits): 32-bit division
      int rr = int(loc);
      int64_t ls = 1;
      for (int k = 0; k < F.n_tan; ++k) {
        li[k] = rr % F.dims[k];
        rr /= F.dims[k];
        lstride[k] = ls;
        ls *= F.dims[k];
      }
    }
    const int ax = F.tan_axis[step];
    const int mm = F.dims[step];
    const double* row = A.Minv[ax] + int64_t(li[step]) * mm;
    double sr = 0.0, si = 0.0;
    // dense row of the 1D inverse in batches whose loads are issued before use
    if (step == 0) {
      int64_t g = int64_t(F.normal_index) * A.fc.stride[F.normal_axis];
      for (int k = 0; k < F.n_tan; ++k)
        if (k != step) g += int64_t(li[k]) * A.fc.stride[F.tan_axis[k]];
      const int64_t sg = A.fc.stride[ax];
      for (int jb = 0; jb < mm; jb += kLiftBatch) {
        int pj[kLiftBatch];
        double c[kLiftBatch];
#pragma unroll
        for (int u = 0; u < kLiftBatch; ++u) {
          const int j = min(jb + u, mm - 1);
          pj[u] = A.pos[g + j * sg];
          c[u] = jb + u < mm ? row[j] : 0.0;
        }
        double2 v[kLiftBatch];
#pragma unroll
        for (int u = 0; u < kLiftBatch; ++u) v[u] = r[pj[u]];
#pragma unroll
        for (int u = 0; u < kLiftBatch; ++u) {
          sr = fma(c[u], v[u].x, sr);
          si = fma(c[u], v[u].y, si);
        }
      }
    } else {
      const double2* src = in + F.offset + (loc - int64_t(li[step]) * lstride[step]);
      for (int jb = 0; jb < mm; jb += kLiftBatch) {
        double c[kLiftBatch];
        double2 v[kLiftBatch];
#pragma unroll
        for (int u = 0; u < kLiftBatch; ++u) {
          const int j = min(jb + u, mm - 1);
          c[u] = jb + u < mm ? row[j] : 0.0;
          v[u] = src[j * lstride[step]];
        }
#pragma unroll
        for (int u = 0; u < kLiftBatch; ++u) {
          sr = fma(c[u], v[u].x, sr);
          si = fma(c[u], v[u].y, si);
        }
      }
    }
    out[e] = make_double2(sr, si);
  }
}

// z[i] = sum over the faces containing i of the packed face result; partials of <r,r> and <r,z>.
__global__ void __launch_bounds__(256) lift_prec_sum_kernel(LiftArgs A, const double2* __restrict__ W,
                                                            const double2* __restrict__ r, double2* __restrict__ z,
                                                            double* __restrict__ part_rr,
                                                            double* __restrict__ part_rz,
                                                            const LiftState* __restrict__ st) {
  __shared__ double lds[4];
  if (st->done) return;
  double arr = 0.0, arz = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < A.n_fixed; i += int64_t(gridDim.x) * blockDim.x) {
    int idx[4];
    fixed_index(A, i, idx);
    double zr = 0.0, zi = 0.0;
    for (int f = 0; f < A.fc.count; ++f) {
      const LiftFace& F = A.fc.f[f];
      if (idx[F.normal_axis] != F.normal_index) continue;
      int64_t loc = 0, ls = 1;
      for (int k = 0; k < F.n_tan; ++k) {
        loc += int64_t(idx[F.tan_axis[k]]) * ls;
        ls *= F.dims[k];
      }
      const double2 v = W[F.offset + loc];
      zr += v.x;
      zi += v.y;
    }
    z[i] = make_double2(zr, zi);
    const double2 rv = r[i];
    arr += rv.x * rv.x + rv.y * rv.y;
    arz += rv.x * zr + rv.y * zi;
  }
  const double t1 = block_sum256(arr, lds);
  const double t2 = block_sum256(arz, lds);
  if (threadIdx.x == 0) {
    part_rr[blockIdx.x] = t1;
    part_rz[blockIdx.x] = t2;
  }
}

__global__ void __launch_bounds__(256) lift_update_kernel(double2* __restrict__ g, double2* __restrict__ r,
                                                          const double2* __restrict__ p,
                                                          const double2* __restrict__ q, int64_t n,
                                                          const LiftState* __restrict__ st) {
  if (st->done) return;
  const double al = st->alpha;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const double2 pv = p[i], qv = q[i];
    double2 gv = g[i], rv = r[i];
    gv.x = fma(al, pv.x, gv.x);
    gv.y = fma(al, pv.y, gv.y);
    rv.x = fma(-al, qv.x, rv.x);
    rv.y = fma(-al, qv.y, rv.y);
    g[i] = gv;
    r[i] = rv;
  }
}

// p = z + beta p (first: p = z).
__global__ void __launch_bounds__(256) lift_p_kernel(double2* __restrict__ p, const double2* __restrict__ z, int64_t n,
                                                     const LiftState* __restrict__ st, int first) {
  if (!first && st->done) return;
  const double be = first ? 0.0 : st->beta;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const double2 zv = z[i];
    if (first) {
      p[i] = zv;
    } else {
      const double2 pv = p[i];
      p[i] = make_double2(fma(be, pv.x, zv.x), fma(be, pv.y, zv.y));
    }
  }
}

enum { LIFT_RESET = 0, LIFT_INIT = 1, LIFT_ALPHA = 2, LIFT_BETA = 3 };

// Scalar step of the lifting CG (one block of kLiftScalarThreads; thread 0 updates the state).
constexpr int kLiftScalarThreads = 256;
__global__ void __launch_bounds__(kLiftScalarThreads) lift_scalar_kernel(int mode, const double* __restrict__ pa,
                                                                         const double* __restrict__ pb, int nparts,
                                                                         LiftState* __restrict__ st,
                                                                         int* __restrict__ status_out, int max_iter) {
  __shared__ double red[2][kLiftScalarThreads / 64];
  if (blockIdx.x != 0) return;
  // partial sums: thread l adds the partials l, l + T, ... (in batches of 8 loads: the matvec's
  // few thousand partials in three memory round trips), then a fixed-order block reduction
  constexpr int T = kLiftScalarThreads;
  double a = 0.0, b = 0.0;
  for (int k0 = 0; k0 < nparts; k0 += T * 8) {
    double va[8], vb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = k0 + u * T + int(threadIdx.x);
      va[u] = (pa && k < nparts) ? pa[k] : 0.0;
      vb[u] = (pb && k < nparts) ? pb[k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a += va[u];
      b += vb[u];
    }
  }
  a = wave_sum64(a);
  b = wave_sum64(b);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  a = 0.0;
  b = 0.0;
  for (int w = 0; w < T / 64; ++w) {
    a += red[0][w];
    b += red[1][w];
  }
  LiftState s = *st;
  if (mode == LIFT_RESET) {
    s.bn = s.rz = s.alpha = s.beta = s.rn = 0.0;
    s.done = 0;
    s.iters = 0;
  } else if (mode == LIFT_INIT) {
    s.bn = a;
    s.rz = b;
    s.rn = a;
    s.iters = 0;
    s.done = (a == 0.0) ? 1 : 0;
    if (!(b > 0.0) && a != 0.0) s.done = 2;
  } else if (mode == LIFT_ALPHA) {
    if (s.done) return;
    if (!(a > 0.0) || !isfinite(a)) {
      s.done = 2;
    } else {
      s.alpha = s.rz / a;
    }
  } else {
    if (s.done) return;
    s.iters += 1;
    s.rn = a;
    if (!isfinite(a) || !isfinite(b)) {
      s.done = 2;
    } else if (a <= kLiftTol2 * s.bn) {
      s.done = 1;
    } else if (!(b > 0.0)) {
      s.done = 2;
    } else if (s.iters >= max_iter) {
      s.done = 3;
    } else {
      s.beta = b / s.rz;
      s.rz = b;
    }
  }
  *st = s;
  if (status_out) status_out[0] = s.done;
}

// b[pos[g(F, loc)]] += loc_vals[loc] for the entries of one face (entries of a face are distinct).
__global__ void __launch_bounds__(256) lift_face_scatter_kernel(LiftArgs A, int f, const double2* __restrict__ vals,
                                                                double2* __restrict__ b) {
  const LiftFace& F = A.fc.f[f];
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < F.size; e += int64_t(gridDim.x) * blockDim.x) {
    int64_t rr = e, g = int64_t(F.normal_index) * A.fc.stride[F.normal_axis];
    for (int k = 0; k < F.n_tan; ++k) {
      g += (rr % F.dims[k]) * A.fc.stride[F.tan_axis[k]];
      rr /= F.dims[k];
    }
    const int64_t i = A.pos[g];
    double2 v = b[i];
    const double2 w = vals[e];
    v.x += w.x;
    v.y += w.y;
    b[i] = v;
  }
}

// G (full tensor) = 0 except G[fixed[i]] = g[i].
__global__ void __launch_bounds__(256) lift_expand_kernel(const double2* __restrict__ gv, const int* __restrict__ pos,
                                                          double2* __restrict__ G, int64_t n_full) {
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n_full; k += int64_t(gridDim.x) * blockDim.x) {
    const int i = pos[k];
    G[k] = (i >= 0) ? gv[i] : make_double2(0.0, 0.0);
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {

// Dense inverse of a symmetric positive definite m x m matrix (Cholesky, then C^{-T} C^{-1}).
bool spd_inverse(const std::vector<double>& M, int m, std::vector<double>& inv) {
  std::vector<double> C(size_t(m) * m, 0.0);
  for (int j = 0; j < m; ++j) {
    double s = M[size_t(j) * m + j];
    for (int k = 0; k < j; ++k) s -= C[size_t(j) * m + k] * C[size_t(j) * m + k];
    if (!(s > 0.0)) return false;
    const double cjj = std::sqrt(s);
    C[size_t(j) * m + j] = cjj;
    for (int i = j + 1; i < m; ++i) {
      double t = M[size_t(i) * m + j];
      for (int k = 0; k < j; ++k) t -= C[size_t(i) * m + k] * C[size_t(j) * m + k];
      C[size_t(i) * m + j] = t / cjj;
    }
  }
  // X = C^{-1} (lower triangular), inv = X^T X
  std::vector<double> X(size_t(m) * m, 0.0);
  for (int c = 0; c < m; ++c)
    for (int i = c; i < m; ++i) {
      double t = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) t -= C[size_t(i) * m + k] * X[size_t(k) * m + c];
      X[size_t(i) * m + c] = t / C[size_t(i) * m + i];
    }
  inv.assign(size_t(m) * m, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      double t = 0.0;
      for (int k = std::max(i, j); k < m; ++k) t += X[size_t(k) * m + i] * X[size_t(k) * m + j];
      inv[size_t(i) * m + j] = t;
    }
  return true;
}

LiftArgs lift_args(const LoadPlan& plan) {
  LiftArgs A;
  A.fc = plan.faces;
  A.fixed = plan.fixed;
  A.fixed_idx = plan.fixed_idx;
  A.pos = plan.pos;
  A.n_fixed = plan.n_fixed;
  for (int a = 0; a < 4; ++a) {
    A.Mband[a] = plan.Mband[a];
    A.Minv[a] = plan.Minv[a];
  }
  return A;
}

struct RhsWork {
  double *R, *A0, *A2, *T0, *T1, *F0, *F1, *g, *r, *z, *p, *q, *W0, *W1, *part;
  LiftState* st;
};

size_t work_layout(const LoadPlan& plan, RhsWork* w, double* base) {
  size_t grid = 1, mid = size_t(plan.m[0]), fmax = 1;
  for (int a = 0; a < plan.na; ++a) grid *= size_t(plan.Q[a]);
  for (int a = 1; a < plan.na; ++a) mid *= size_t(std::max(plan.m[a], plan.Q[a]));
  for (int f = 0; f < plan.faces.count; ++f) {
    size_t s = 1;
    for (int k = 0; k < plan.faces.f[f].n_tan; ++k) {
      const int ax = plan.faces.f[f].tan_axis[k];
      s *= size_t(std::max(plan.m[ax], plan.Q[ax]));
    }
    fmax = std::max(fmax, s);
  }
  const size_t nf = size_t(plan.n_fixed), tot = size_t(plan.faces.total);
  // partial sums: two per fixed-set block (preconditioner), one per lifting-matvec block
  const size_t nparts = std::max(2 * size_t(std::max(plan.lift_blocks, 1)),
                                 size_t((plan.n_fixed + kLiftMvWaves - 1) / kLiftMvWaves) + 1);
  size_t off = 0;
  auto take = [&](double** dst, size_t n) {
    if (w) *dst = base + off;
    off += (n + 31) & ~size_t(31);  // 256-byte aligned sub-buffers
  };
  RhsWork dummy;
  RhsWork* ww = w ? w : &dummy;
  take(&ww->R, 2 * grid);
  take(&ww->A0, 2 * mid);
  take(&ww->A2, 2 * mid);
  take(&ww->T0, 2 * mid);
  take(&ww->T1, 2 * mid);
  take(&ww->F0, 2 * fmax);
  take(&ww->F1, 2 * fmax);
  take(&ww->g, 2 * nf);
  take(&ww->r, 2 * nf);
  take(&ww->z, 2 * nf);
  take(&ww->p, 2 * nf);
  take(&ww->q, 2 * nf);
  take(&ww->W0, 2 * tot);
  take(&ww->W1, 2 * tot);
  take(&ww->part, nparts);
  double* stp = nullptr;
  take(&stp, 8);
  if (w) w->st = reinterpret_cast<LiftState*>(stp);
  return off;
}

}  // namespace

int load_plan_build(const HostProblem& hp, LoadPlan& plan) {
  plan.na = hp.d + 1;
  const Direction* dirs[4] = {&hp.dir_t, &hp.dir_s[0], &hp.dir_s[1], &hp.dir_s[2]};
  const std::vector<double>* mfull[4] = {&hp.Mfull_t, &hp.Mfull_s[0], &hp.Mfull_s[1], &hp.Mfull_s[2]};
  LiftFaces& fc = plan.faces;
  fc.na = plan.na;
  int64_t stride = 1;
  for (int a = 0; a < plan.na; ++a) {
    const Direction& D = *dirs[a];
    const int Q = int(D.x.size()), m = D.m, p = D.p;
    const int n = (a == 0) ? m - 1 : m - 2;
    plan.Q[a] = Q;
    plan.m[a] = m;
    plan.n[a] = n;
    fc.m[a] = m;
    fc.p[a] = p;
    fc.stride[a] = stride;
    stride *= m;
    std::vector<int> elo(Q), ehi(Q), llo(n, Q), lhi(n, 0), wlo(m, Q), whi(m, 0);
    std::vector<double> ev[3], ld[3], wf(size_t(m) * Q, 0.0);
    for (int r = 0; r < 3; ++r) {
      ev[r].assign(size_t(Q) * m, 0.0);
      ld[r].assign(size_t(n) * Q, 0.0);
    }
    for (int e = 0; e < D.n_el; ++e)
      for (int g = 0; g < D.q; ++g) {
        const int q = e * D.q + g;
        elo[q] = D.first[e];
        ehi[q] = D.first[e] + p + 1;
        for (int k = 0; k <= p; ++k) {
          const int i = D.first[e] + k;
          for (int r = 0; r < 3; ++r) ev[r][size_t(q) * m + i] = D.b(e, g, r, k);
          wf[size_t(i) * Q + q] = D.w[q] * D.b(e, g, 0, k);
          wlo[i] = std::min(wlo[i], q);
          whi[i] = std::max(whi[i], q + 1);
          // free index: the first function dropped (space; time of the least-squares method) or
          // the last one (time of the ultraweak method)
          const int fi = (a == 0 && hp.time_final) ? i : i - 1;
          if (fi < 0 || fi >= n) continue;
          for (int r = 0; r < 3; ++r) ld[r][size_t(fi) * Q + q] = D.w[q] * D.b(e, g, r, k);
          llo[fi] = std::min(llo[fi], q);
          lhi[fi] = std::max(lhi[fi], q + 1);
        }
      }
    for (int r = 0; r < 3; ++r) {
      if (int rc = plan_upload(plan, &plan.eval[a][r], ev[r])) return rc;
      if (int rc = plan_upload(plan, &plan.load[a][r], ld[r])) return rc;
    }
    if (int rc = plan_upload(plan, &plan.eval_lo[a], elo)) return rc;
    if (int rc = plan_upload(plan, &plan.eval_hi[a], ehi)) return rc;
    if (a == 0) {
      // time axis: the bands of the evaluation (rows q) and load (rows i) matrices transposed,
      // band[u][row] = M[row][lo_row + u], so that the rows of consecutive threads are adjacent
      int ew = 0, lw = 0;
      for (int q = 0; q < Q; ++q) ew = std::max(ew, ehi[q] - elo[q]);
      for (int i = 0; i < n; ++i) lw = std::max(lw, lhi[i] - llo[i]);
      plan.tband_ew = ew;
      plan.tband_lw = lw;
      for (int r = 0; r < 2; ++r) {
        std::vector<double> eb(size_t(ew) * Q, 0.0), lb(size_t(std::max(lw, 1)) * n, 0.0);
        for (int q = 0; q < Q; ++q)
          for (int u = 0; u < ehi[q] - elo[q]; ++u) eb[size_t(u) * Q + q] = ev[r][size_t(q) * m + elo[q] + u];
        for (int i = 0; i < n; ++i)
          for (int u = 0; u < lhi[i] - llo[i]; ++u) lb[size_t(u) * n + i] = ld[r][size_t(i) * Q + llo[i] + u];
        if (int rc = plan_upload(plan, &plan.tband_eval[r], eb)) return rc;
        if (int rc = plan_upload(plan, &plan.tband_load[r], lb)) return rc;
      }
    }
    if (int rc = plan_upload(plan, &plan.load_lo[a], llo)) return rc;
    if (int rc = plan_upload(plan, &plan.load_hi[a], lhi)) return rc;
    if (int rc = plan_upload(plan, &plan.wfull[a], wf)) return rc;
    if (int rc = plan_upload(plan, &plan.wfull_lo[a], wlo)) return rc;
    if (int rc = plan_upload(plan, &plan.wfull_hi[a], whi)) return rc;
    // banded and inverse full mass matrices
    const std::vector<double>& M = *mfull[a];
    std::vector<double> band(size_t(m) * (2 * p + 1), 0.0), inv;
    for (int i = 0; i < m; ++i)
      for (int j = std::max(0, i - p); j <= std::min(m - 1, i + p); ++j)
        band[size_t(i) * (2 * p + 1) + (j - i + p)] = M[size_t(i) * m + j];
    if (!spd_inverse(M, m, inv)) return -2;
    if (int rc = plan_upload(plan, &plan.Mband[a], band)) return rc;
    if (int rc = plan_upload(plan, &plan.Minv[a], inv)) return rc;
  }
  plan.n_full = stride;
  // faces: initial (time index 0), then x_l = 0 and x_l = 1
  fc.count = 0;
  auto add_face = [&](int axis, int index) {
    LiftFace& F = fc.f[fc.count++];
    F.normal_axis = axis;
    F.normal_index = index;
    F.n_tan = 0;
    F.size = 1;
    for (int a = 0; a < plan.na; ++a)
      if (a != axis) {
        F.tan_axis[F.n_tan] = a;
        F.dims[F.n_tan] = fc.m[a];
        F.size *= fc.m[a];
        ++F.n_tan;
      }
  };
  add_face(0, 0);
  for (int l = 1; l < plan.na; ++l) {
    add_face(l, 0);
    add_face(l, fc.m[l] - 1);
  }
  fc.total = 0;
  for (int f = 0; f < fc.count; ++f) {
    fc.f[f].offset = fc.total;
    fc.total += fc.f[f].size;
  }
  std::vector<int> pos(size_t(plan.n_full), -1);
  std::vector<int64_t> fixed;
  for (int f = 0; f < fc.count; ++f) {
    const LiftFace& F = fc.f[f];
    for (int64_t e = 0; e < F.size; ++e) {
      int64_t rr = e, g = int64_t(F.normal_index) * fc.stride[F.normal_axis];
      for (int k = 0; k < F.n_tan; ++k) {
        g += (rr % F.dims[k]) * fc.stride[F.tan_axis[k]];
        rr /= F.dims[k];
      }
      if (pos[size_t(g)] < 0) {
        pos[size_t(g)] = int(fixed.size());
        fixed.push_back(g);
      }
    }
  }
  plan.n_fixed = int64_t(fixed.size());
  plan.lift_blocks = int(std::min<int64_t>((plan.n_fixed + 255) / 256, 1024));
  std::vector<int> fixed_idx(size_t(plan.n_fixed) * 4, 0);
  for (size_t i = 0; i < fixed.size(); ++i)
    for (int a = 0; a < fc.na; ++a) fixed_idx[i * 4 + a] = int((fixed[i] / fc.stride[a]) % fc.m[a]);
  if (int rc = plan_upload(plan, &plan.fixed, fixed)) return rc;
  if (int rc = plan_upload(plan, &plan.fixed_idx, fixed_idx)) return rc;
  if (int rc = plan_upload(plan, &plan.pos, pos)) return rc;
  return 0;
}

void load_plan_free(LoadPlan& plan) {
  for (void* p : plan.allocs) (void)hipFree(p);
  plan.allocs.clear();
}

size_t rhs_work_reals(const LoadPlan& plan) { return work_layout(plan, nullptr, nullptr); }

namespace {

// u_bar: b from the face data, then preconditioned CG on the fixed set, then G.
int lifting_device(const LoadPlan& plan, const double* u0_q, const double* const* faces, double* G,
                   const RhsWork& w, int* status_dev, volatile int* status_host, int max_iter, hipStream_t s) {
  const LiftArgs A = lift_args(plan);
  const int64_t nf = plan.n_fixed;
  const int nb = plan.lift_blocks;
  int rc;
  const int64_t mvb = (nf + kLiftMvWaves - 1) / kLiftMvWaves;  // lifting-matvec blocks (one partial each)
  auto scalar = [&](int mode, const double* pa, const double* pb, int nparts = 0) -> int {
    hipLaunchKernelGGL(lift_scalar_kernel, dim3(1), dim3(kLiftScalarThreads), 0, s, mode, pa, pb,
                       nparts > 0 ? nparts : nb, w.st, status_dev, max_iter);
    return int(hipGetLastError());
  };
  if ((rc = scalar(LIFT_RESET, nullptr, nullptr))) return rc;
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(2 * nf)), dim3(256), 0, s, w.r, 2 * nf);
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(2 * nf)), dim3(256), 0, s, w.g, 2 * nf);
  if ((rc = int(hipGetLastError()))) return rc;
  // b_F = face data contracted with the weighted full basis along the tangent axes
  for (int f = 0; f < plan.faces.count; ++f) {
    const double* data = (f == 0) ? u0_q : (faces ? faces[f - 1] : nullptr);
    if (!data) continue;
    const LiftFace& F = plan.faces.f[f];
    Shape sh;
    sh.na = F.n_tan;
    for (int k = 0; k < F.n_tan; ++k) sh.dims[k] = plan.Q[F.tan_axis[k]];
    const double* src = data;
    double* buf[2] = {w.F0, w.F1};
    for (int k = 0; k < F.n_tan; ++k) {
      const int ax = F.tan_axis[k];
      double* o = buf[k & 1];
      if ((rc = contract(src, o, sh, k, plan.wfull[ax], plan.wfull_lo[ax], plan.wfull_hi[ax], plan.Q[ax], plan.m[ax],
                         1.0, 0.0, false, s)))
        return rc;
      src = o;
    }
    hipLaunchKernelGGL(lift_face_scatter_kernel, dim3(grid_for(F.size)), dim3(256), 0, s, A, f,
                       (const double2*)src, (double2*)w.r);
    if ((rc = int(hipGetLastError()))) return rc;
  }
  // z = sum_F P_F^T M_F^{-1} P_F r with partials of <r,r> and <r,z>
  auto precondition = [&]() -> int {
    const double* in = nullptr;
    double* bufs[2] = {w.W0, w.W1};
    const int nt = plan.faces.f[0].n_tan;
    for (int k = 0; k < nt; ++k) {
      hipLaunchKernelGGL(lift_prec_axis_kernel, dim3(grid_for(plan.faces.total)), dim3(256), 0, s, A, k,
                         (const double2*)w.r, (const double2*)in, (double2*)bufs[k & 1], (const LiftState*)w.st);
      in = bufs[k & 1];
    }
    hipLaunchKernelGGL(lift_prec_sum_kernel, dim3(nb), dim3(256), 0, s, A, (const double2*)in, (const double2*)w.r,
                       (double2*)w.z, w.part, w.part + nb, (const LiftState*)w.st);
    return int(hipGetLastError());
  };
  if ((rc = precondition())) return rc;
  if ((rc = scalar(LIFT_INIT, w.part, w.part + nb))) return rc;
  hipLaunchKernelGGL(lift_p_kernel, dim3(grid_for(nf)), dim3(256), 0, s, (double2*)w.p, (const double2*)w.z, nf,
                     (const LiftState*)w.st, 1);
  if ((rc = int(hipGetLastError()))) return rc;
  // iterations in chunks; the host checks the device's status after each chunk
  constexpr int kChunk = 4;
  for (int it = 0; it < max_iter; it += kChunk) {
    for (int c = 0; c < kChunk; ++c) {
      hipLaunchKernelGGL(lift_matvec_kernel, dim3(static_cast<unsigned>(mvb)), dim3(64 * kLiftMvWaves), 0, s, A,
                         (const double2*)w.p, (double2*)w.q, w.part, (const LiftState*)w.st);
      if ((rc = int(hipGetLastError()))) return rc;
      if ((rc = scalar(LIFT_ALPHA, w.part, nullptr, int(mvb)))) return rc;
      hipLaunchKernelGGL(lift_update_kernel, dim3(grid_for(nf)), dim3(256), 0, s, (double2*)w.g, (double2*)w.r,
                         (const double2*)w.p, (const double2*)w.q, nf, (const LiftState*)w.st);
      if ((rc = int(hipGetLastError()))) return rc;
      if ((rc = precondition())) return rc;
      if ((rc = scalar(LIFT_BETA, w.part, w.part + nb))) return rc;
      hipLaunchKernelGGL(lift_p_kernel, dim3(grid_for(nf)), dim3(256), 0, s, (double2*)w.p, (const double2*)w.z, nf,
                         (const LiftState*)w.st, 0);
      if ((rc = int(hipGetLastError()))) return rc;
    }
    if ((rc = int(hipStreamSynchronize(s)))) return rc;
    if (*status_host != 0) break;
  }
  hipLaunchKernelGGL(lift_expand_kernel, dim3(grid_for(plan.n_full)), dim3(256), 0, s, (const double2*)w.g, plan.pos,
                     (double2*)G, plan.n_full);
  return int(hipGetLastError());
}

// f_bar = (f - S_V u_bar, S_V B_I) by sum factorisation (see the top of this file).  On a
// mapped domain the Laplacian is sum_k c_k D^k and every spatial integral carries J.
int load_vector_device(const HostProblem& hp, const LoadPlan& plan, const double* f_q, const double* G, double* fbar,
                       const RhsWork& w, hipStream_t s) {
  const int na = plan.na;
  const double nu = hp.nu;
  size_t grid = 1;
  for (int a = 0; a < na; ++a) grid *= size_t(plan.Q[a]);
  double* R = w.R;
  double* A0 = w.A0;
  double* A2 = w.A2;
  double* T[2] = {w.T0, w.T1};
  int rc;

  // evaluation on the grid: chain over the spatial axes with derivative order ord[l] on x_l
  auto eval_chain = [&](const int* ord, double* dst, bool accumulate, double ar) -> int {
    Shape sh;
    sh.na = na;
    for (int a = 0; a < na; ++a) sh.dims[a] = plan.m[a];
    const double* src = G;
    for (int a = 1; a < na; ++a) {
      const bool last = (a == na - 1);
      double* o = last ? dst : T[a & 1];
      const int r = ord ? ord[a - 1] : 0;
      int e = contract(src, o, sh, a, plan.eval[a][r], plan.eval_lo[a], plan.eval_hi[a], plan.m[a], plan.Q[a],
                       last ? ar : 1.0, 0.0, last && accumulate, s);
      if (e) return e;
      src = o;
    }
    return 0;
  };
  const int64_t mid_t = int64_t(plan.m[0]);
  int64_t msz = mid_t;
  for (int a = 1; a < na; ++a) msz *= plan.Q[a];
  if ((rc = eval_chain(nullptr, A0, false, 1.0))) return rc;
  // A2 = nu Lap u_bar
  for (int k = 0; k < plan.n_lap; ++k) {
    if (!plan.lap_c[k]) {
      if ((rc = eval_chain(plan.lap_ord[k], A2, k > 0, nu))) return rc;
    } else {
      if ((rc = eval_chain(plan.lap_ord[k], R, false, 1.0))) return rc;
      hipLaunchKernelGGL(scale_add_kernel, dim3(grid_for(msz)), dim3(256), 0, s, (const double2*)R, plan.lap_c[k],
                         (double2*)A2, mid_t, msz, nu, k > 0 ? 1 : 0);
      if ((rc = int(hipGetLastError()))) return rc;
    }
  }
  // C = nu Lap u_bar - V u_bar (in place in A2), per spatial point, time fastest
  if (plan.Vq) {
    hipLaunchKernelGGL(combine_v_kernel, dim3(grid_for(msz)), dim3(256), 0, s, (const double2*)A2,
                       (const double2*)A0, plan.Vq, (const double*)nullptr, (double2*)A2, mid_t, msz, 1.0, 0.0,
                       -1.0);
    if ((rc = int(hipGetLastError()))) return rc;
  }
  // R = f - i B_t'^T A0 + B_t^T C, then X0 = B_t^w R and Y = J (-i B_t'^w R + V X0) (in X1) for the
  // free time rows: one pass each over the space-time grid, one block per spatial grid point
  double* X0 = A0;
  double* X1 = A2;
  double* S = R;  // scratch for the c_k J X0 products below
  int64_t xs = plan.n[0];
  {
    int64_t npts = 1;
    for (int a = 1; a < na; ++a) npts *= plan.Q[a];
    const int m0 = plan.m[0], Q0 = plan.Q[0], n0 = plan.n[0];
    const size_t fused_lds = (2 * size_t(m0) + size_t(Q0)) * sizeof(double2);
    if (fused_lds <= kTimeRhsMaxLds && 2 * n0 <= Q0) {
      // one launch, R kept in LDS: X0 and X1 go to the (unused) R buffer, since a block's outputs
      // would overwrite inputs of other blocks in A0 and A2; A0 is then the scratch
      X0 = R;
      X1 = R + 2 * int64_t(n0) * npts;
      S = A0;
      if ((rc = allow_lds(reinterpret_cast<const void*>(&time_rhs_kernel), fused_lds))) return rc;
      hipLaunchKernelGGL(time_rhs_kernel, dim3(static_cast<unsigned>(npts)), dim3(256), fused_lds, s,
                         (const double2*)A0, (const double2*)A2, (const double2*)f_q, plan.tband_eval[0],
                         plan.tband_eval[1], plan.eval_lo[0], plan.tband_ew, m0, Q0, (double2*)X0, (double2*)X1,
                         plan.tband_load[0], plan.tband_load[1], plan.load_lo[0], plan.tband_lw, n0, plan.Vq,
                         plan.Jq);
      if ((rc = int(hipGetLastError()))) return rc;
    } else {
      if ((rc = allow_lds(reinterpret_cast<const void*>(&time_expand_kernel), 2 * m0 * sizeof(double2))) ||
          (rc = allow_lds(reinterpret_cast<const void*>(&time_load_kernel), Q0 * sizeof(double2))))
        return rc;
      hipLaunchKernelGGL(time_expand_kernel, dim3(static_cast<unsigned>(npts)), dim3(256), 2 * m0 * sizeof(double2),
                         s, (const double2*)A0, (const double2*)A2, (const double2*)f_q, (double2*)R,
                         plan.tband_eval[0], plan.tband_eval[1], plan.eval_lo[0], plan.tband_ew, m0, Q0);
      if ((rc = int(hipGetLastError()))) return rc;
      hipLaunchKernelGGL(time_load_kernel, dim3(static_cast<unsigned>(npts)), dim3(128), Q0 * sizeof(double2), s,
                         (const double2*)R, (double2*)X0, (double2*)X1, plan.tband_load[0], plan.tband_load[1],
                         plan.load_lo[0], plan.tband_lw, Q0, n0, plan.Vq, plan.Jq);
      if ((rc = int(hipGetLastError()))) return rc;
    }
    xs *= npts;
  }
  auto load_chain = [&](const double* src0, const int* ord, double ar, bool accumulate) -> int {
    Shape sh;
    sh.na = na;
    sh.dims[0] = plan.n[0];
    for (int a = 1; a < na; ++a) sh.dims[a] = plan.Q[a];
    const double* src = src0;
    for (int a = 1; a < na; ++a) {
      const bool last = (a == na - 1);
      double* o = last ? fbar : T[a & 1];
      const int r = ord ? ord[a - 1] : 0;
      int e = contract(src, o, sh, a, plan.load[a][r], plan.load_lo[a], plan.load_hi[a], plan.Q[a], plan.n[a],
                       last ? ar : 1.0, 0.0, last && accumulate, s);
      if (e) return e;
      src = o;
    }
    return 0;
  };
  if ((rc = load_chain(X1, nullptr, 1.0, false))) return rc;
  // - nu sum_k (D^k phi_I, c_k J X0): the scratch S holds c_k J X0
  for (int k = 0; k < plan.n_lap; ++k) {
    const double* src = X0;
    if (plan.lap_cJ[k]) {
      hipLaunchKernelGGL(scale_add_kernel, dim3(grid_for(xs)), dim3(256), 0, s, (const double2*)X0, plan.lap_cJ[k],
                         (double2*)S, int64_t(plan.n[0]), xs, 1.0, 0);
      if ((rc = int(hipGetLastError()))) return rc;
      src = S;
    }
    if ((rc = load_chain(src, plan.lap_ord[k], -nu, true))) return rc;
  }
  return 0;
}

}  // namespace

// X0[o][0] += i u0[o] for every spatial grid point o (time row 0 of the free basis of W_h: the
// only time function that is non-zero at t = 0, where it equals 1)
__global__ void __launch_bounds__(256) uw_initial_kernel(const double2* __restrict__ u0, double2* __restrict__ X0,
                                                         int64_t npts, int n_t) {
  const int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (o >= npts) return;
  const double2 u = u0[o];
  double2 x = X0[o * n_t];
  x.x -= u.y;  // + i (u.x + i u.y)
  x.y += u.x;
  X0[o * n_t] = x;
}

int ultraweak_rhs_device(const HostProblem& hp, const LoadPlan& plan, const double* f_q, const double* u0_q,
                         double* fbar, double* work, hipStream_t s) {
  (void)hp;
  RhsWork w;
  work_layout(plan, &w, work);
  const int na = plan.na;
  int64_t npts = 1;
  for (int a = 1; a < na; ++a) npts *= plan.Q[a];
  const int Q0 = plan.Q[0], n0 = plan.n[0];
  double* X0 = w.A0;
  int rc;
  // time: X0[o][i_t] = sum_q w_q b_{i_t}(t_q) f(t_q, x_o) (free time rows of W_h)
  if (f_q) {
    if ((rc = allow_lds(reinterpret_cast<const void*>(&time_load_kernel), Q0 * sizeof(double2)))) return rc;
    hipLaunchKernelGGL(time_load_kernel, dim3(static_cast<unsigned>(npts)), dim3(128), Q0 * sizeof(double2), s,
                       (const double2*)f_q, (double2*)X0, (double2*)w.A2, plan.tband_load[0], plan.tband_load[1],
                       plan.load_lo[0], plan.tband_lw, Q0, n0, (const double*)nullptr, (const double*)nullptr);
  } else {
    hipLaunchKernelGGL(zero_kernel, dim3(grid_for(2 * npts * n0)), dim3(256), 0, s, X0, 2 * npts * n0);
  }
  if ((rc = int(hipGetLastError()))) return rc;
  if (u0_q) {
    hipLaunchKernelGGL(uw_initial_kernel, dim3(unsigned((npts + 255) / 256)), dim3(256), 0, s, (const double2*)u0_q,
                       (double2*)X0, npts, n0);
    if ((rc = int(hipGetLastError()))) return rc;
  }
  // space: contract every spatial axis with the weighted free functions (order 0)
  Shape sh;
  sh.na = na;
  sh.dims[0] = n0;
  for (int a = 1; a < na; ++a) sh.dims[a] = plan.Q[a];
  double* T[2] = {w.T0, w.T1};
  const double* src = X0;
  for (int a = 1; a < na; ++a) {
    const bool last = (a == na - 1);
    double* o = last ? fbar : T[a & 1];
    if ((rc = contract(src, o, sh, a, plan.load[a][0], plan.load_lo[a], plan.load_hi[a], plan.Q[a], plan.n[a], 1.0,
                       0.0, false, s)))
      return rc;
    src = o;
  }
  return 0;
}

int rhs_device(const HostProblem& hp, const LoadPlan& plan, const double* f_q, const double* u0_q,
               const double* const* faces, double* G, double* fbar, double* work, int* status_dev,
               volatile int* status_host, int max_iter, hipStream_t stream) {
  RhsWork w;
  work_layout(plan, &w, work);
  int rc = lifting_device(plan, u0_q, faces, G, w, status_dev, status_host, max_iter, stream);
  if (rc) return rc;
  return load_vector_device(hp, plan, f_q, G, fbar, w, stream);
}

}  // namespace stfd
