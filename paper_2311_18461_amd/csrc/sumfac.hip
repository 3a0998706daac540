// Sum-factorised system matvec (see sumfac.h for the factorisation).
//
// Pass 1 (x_1 and time): one block per (spatial pencil i_2, i_3; segment of x_1 rows), one thread
//   per time index; the segment's rows of X (and a halo of p_s rows) are staged in LDS, and each
//   thread walks the rows with a register window of the time products L_t X, i K_t X, M_t X.
// Middle pass (x_2, d = 3) and last pass (x_2 for d = 2, x_3 for d = 3): one thread per line along
//   the axis and segment of rows (consecutive lanes on consecutive lines, so every load of a wave
//   is contiguous), with a sliding window of 2 p_s + 1 rows per input in registers.
// The last pass also writes one partial of Re <x, y> per block (PCG's <p, A p>).
#include "sumfac.h"

#include <algorithm>
#include <cmath>

namespace stfd {

constexpr int kSfBlock = 256;
constexpr int kSfSeg = 12;     // rows per thread of an axis pass (about: the same length for all)
constexpr int kSfSegMax = 24;  // longest segment (LDS of the band rows)

struct SfPass1Args {
  const double2* x;
  double2* za;
  double2* zb;
  double2* zc;
  const double* band;   // direction x_1: [3][n1][2 ps + 1]
  const double* tband;  // [n_t][2 pt + 1][4]
  int n1, n_t, seg, segs;
  int64_t N;            // complex entries per right-hand side
  const int* done;
};

// One block per (spatial pencil i_2, i_3; segment of x_1 rows); thread t owns time index t.  The
// segment's rows of X and their 2 ps halo rows are staged in LDS with one batch of loads, the time
// band rows of t stay in registers, and the thread walks the segment keeping the time products
// (L_t X, i K_t X, M_t X) of the 2 ps + 1 rows around the current one in registers: each row's
// products are formed once, when it enters the window.
template <int PS, int PT>
__global__ __launch_bounds__(128) void sf_pass1_kernel(SfPass1Args a) {
  extern __shared__ __align__(16) unsigned char sf_smem[];
  constexpr int WS = 2 * PS + 1, WT = 2 * PT + 1;
  const int64_t rhs = blockIdx.y;
  if (a.done && a.done[rhs]) return;
  const int64_t pencil = blockIdx.x / a.segs;
  const int sg = int(blockIdx.x - pencil * a.segs);
  const int n1 = a.n1, nt = a.n_t;
  const int r0 = sg * a.seg, r1 = min(r0 + a.seg, n1);        // output rows
  const int w0 = max(r0 - PS, 0), w1 = min(r1 + PS, n1);       // staged rows
  const int nw = w1 - w0;
  const int64_t base = rhs * a.N + pencil * int64_t(n1) * nt;
  const int t = threadIdx.x;
  const int tc = min(t, nt - 1);
  double2* Xs = reinterpret_cast<double2*>(sf_smem);                        // [nw][nt]
  double* Bs = reinterpret_cast<double*>(Xs + int64_t(a.seg + 2 * PS) * nt);  // [3][seg][WS]
  {
    const double2* X = a.x + base + int64_t(w0) * nt;
    for (int j = 0; j < nw; ++j)
      if (t < nt) Xs[j * nt + t] = X[int64_t(j) * nt + t];
    const int nb = (r1 - r0) * WS;
    for (int k = t; k < 3 * nb; k += blockDim.x) {
      const int c = k / nb, rem = k - c * nb;
      Bs[k] = a.band[(int64_t(c) * n1 + r0) * WS + rem];
    }
  }
  // time band row of t: (L_t, M_t, K_t) (zero where t + dt leaves the axis)
  double tl[WT], tm[WT], tk[WT];
  {
    const double2* tb = reinterpret_cast<const double2*>(a.tband) + tc * WT * 2;
#pragma unroll
    for (int k = 0; k < WT; ++k) {
      const double2 lm = tb[2 * k], kk = tb[2 * k + 1];
      tl[k] = lm.x;
      tm[k] = lm.y;
      tk[k] = kk.x;
    }
  }
  __syncthreads();
  // time products of staged row j (clamped into the staged rows: rows off the matrix meet zero band
  // entries)
  auto tprod = [&](int j, double2& wl, double2& wk, double2& wm) {
    const double2* xr = Xs + (min(max(j, w0), w1 - 1) - w0) * nt;
    double lr = 0.0, li = 0.0, mr = 0.0, mi = 0.0, kr = 0.0, ki = 0.0;
#pragma unroll
    for (int k = 0; k < WT; ++k) {
      const double2 xv = xr[min(max(tc + k - PT, 0), nt - 1)];
      lr = fma(tl[k], xv.x, lr);
      li = fma(tl[k], xv.y, li);
      mr = fma(tm[k], xv.x, mr);
      mi = fma(tm[k], xv.y, mi);
      kr = fma(tk[k], xv.x, kr);
      ki = fma(tk[k], xv.y, ki);
    }
    wl = make_double2(lr, li);
    wk = make_double2(-ki, kr);  // i K_t X
    wm = make_double2(mr, mi);
  };
  double2 WL[WS], WK[WS], WM[WS];
#pragma unroll
  for (int k = 0; k < WS - 1; ++k) tprod(r0 - PS + k, WL[k], WK[k], WM[k]);
  const int nb = (r1 - r0) * WS;
  for (int r = r0; r < r1; ++r) {
    tprod(r + PS, WL[WS - 1], WK[WS - 1], WM[WS - 1]);
    const double* Mb = Bs + (r - r0) * WS;
    const double* Gb = Mb + nb;
    const double* Jb = Gb + nb;
    double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0, cr = 0.0, ci = 0.0;
#pragma unroll
    for (int o = 0; o < WS; ++o) {
      const double m = Mb[o], g = Gb[o], h = Jb[o];
      ar = fma(m, WL[o].x, ar);
      ar = fma(g, WK[o].x, ar);
      ar = fma(h, WM[o].x, ar);
      ai = fma(m, WL[o].y, ai);
      ai = fma(g, WK[o].y, ai);
      ai = fma(h, WM[o].y, ai);
      br = fma(m, WK[o].x, br);
      br = fma(2.0 * g, WM[o].x, br);
      bi = fma(m, WK[o].y, bi);
      bi = fma(2.0 * g, WM[o].y, bi);
      cr = fma(m, WM[o].x, cr);
      ci = fma(m, WM[o].y, ci);
    }
    if (t < nt) {
      const int64_t gi = base + int64_t(r) * nt + t;
      a.za[gi] = make_double2(ar, ai);
      a.zb[gi] = make_double2(br, bi);
      a.zc[gi] = make_double2(cr, ci);
    }
#pragma unroll
    for (int k = 0; k < WS - 1; ++k) {
      WL[k] = WL[k + 1];
      WK[k] = WK[k + 1];
      WM[k] = WM[k + 1];
    }
  }
}

struct SfAxisArgs {
  const double2* in[3];
  double2* out[3];      // middle pass: P, Q, R; last pass: out[0] = y
  const double* band;   // this axis: [3][n][2 ps + 1]
  int n;                // size of the axis
  int seg;              // rows of the axis per thread
  int64_t stride;       // complex entries between neighbours along the axis (entries below it)
  int64_t lines;        // (entries above the axis) * stride: one thread per line and segment
  int64_t N;
  const double2* x;     // last pass: the input vector for <x, y> (or nullptr)
  double* partial;      // [rhs][gridDim.x * gridDim.y] or nullptr
  const int* done;
};

// One thread walks `seg` consecutive rows of one line along the axis, holding the 2 ps + 1 rows of
// each input around the current one in registers: every input entry is loaded once per segment
// (plus a 2 ps halo), the next row's loads issued before the current row is computed.  Rows off the
// axis are zeros.  The row index is the same for all lanes (it depends on the segment and the step
// only), so the band entries are uniform loads.
// LAST: y = M in0 + G in1 + Jh in2 (and the <x, y> partial).  Otherwise
// (out0, out1, out2) = (M in0 + G in1 + Jh in2, M in1 + 2 G in2, M in2).
template <int PS, bool LAST>
__global__ __launch_bounds__(kSfBlock) void sf_axis_kernel(SfAxisArgs a) {
  constexpr int WS = 2 * PS + 1;
  __shared__ double red[kSfBlock / 64];
  __shared__ double Bs[3 * kSfSegMax * WS];  // band rows of this segment (LDS reads: no wait on the prefetch)
  const int64_t rhs = blockIdx.z;
  if (a.done && a.done[rhs]) return;
  const int64_t f = int64_t(blockIdx.x) * kSfBlock + threadIdx.x;
  const bool active = f < a.lines;
  const int64_t fc = active ? f : a.lines - 1;
  const int64_t line = fc / a.stride, c = fc - line * a.stride;
  const int64_t base = rhs * a.N + line * a.n * a.stride + c;  // entry of row 0 of this line
  const double2* in0 = a.in[0] + base;
  const double2* in1 = a.in[1] + base;
  const double2* in2 = a.in[2] + base;
  const int n = a.n;
  const int i0 = int(blockIdx.y) * a.seg, i1 = min(i0 + a.seg, n);
  {
    const int nb = (i1 - i0) * WS;
    for (int k = threadIdx.x; k < 3 * nb; k += kSfBlock) {
      const int c = k / nb, rem = k - c * nb;
      Bs[c * kSfSegMax * WS + rem] = a.band[(int64_t(c) * n + i0) * WS + rem];
    }
  }
  __syncthreads();
  // rows off the axis are read at a clamped row: their band entries are zero (a select between a
  // load and a constant would become a flat load through a pointer select)
  auto row_off = [&](int j) -> int64_t { return int64_t(min(max(j, 0), n - 1)) * a.stride; };
  double2 w0[WS], w1[WS], w2[WS];
#pragma unroll
  for (int k = 0; k < WS - 1; ++k) {
    const int64_t off = row_off(i0 - PS + k);
    w0[k] = in0[off];
    w1[k] = in1[off];
    w2[k] = in2[off];
  }
  // the row entering the window at the first step
  double2 n0, n1, n2;
  {
    const int64_t off = row_off(i0 + PS);
    n0 = in0[off];
    n1 = in1[off];
    n2 = in2[off];
  }
  double part = 0.0;
  for (int i = i0; i < i1; ++i) {
    w0[WS - 1] = n0;
    w1[WS - 1] = n1;
    w2[WS - 1] = n2;
    {
      // prefetch the row entering at the next step (past the segment: a harmless clamped row)
      const int64_t off = row_off(i + PS + 1);
      n0 = in0[off];
      n1 = in1[off];
      n2 = in2[off];
    }
    double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0, cr = 0.0, ci = 0.0;
#pragma unroll
    for (int o = 0; o < WS; ++o) {
      const int bx = (i - i0) * WS + o;
      const double m = Bs[bx], g = Bs[kSfSegMax * WS + bx], h = Bs[2 * kSfSegMax * WS + bx];
      ar = fma(m, w0[o].x, ar);
      ar = fma(g, w1[o].x, ar);
      ar = fma(h, w2[o].x, ar);
      ai = fma(m, w0[o].y, ai);
      ai = fma(g, w1[o].y, ai);
      ai = fma(h, w2[o].y, ai);
      if constexpr (!LAST) {
        br = fma(m, w1[o].x, br);
        br = fma(2.0 * g, w2[o].x, br);
        bi = fma(m, w1[o].y, bi);
        bi = fma(2.0 * g, w2[o].y, bi);
        cr = fma(m, w2[o].x, cr);
        ci = fma(m, w2[o].y, ci);
      }
    }
    const int64_t e = base + int64_t(i) * a.stride;
    if (active) {
      a.out[0][e] = make_double2(ar, ai);
      if constexpr (LAST) {
        if (a.partial) {
          const double2 xv = a.x[e];
          part += xv.x * ar + xv.y * ai;  // Re(conj(x) y)
        }
      } else {
        a.out[1][e] = make_double2(br, bi);
        a.out[2][e] = make_double2(cr, ci);
      }
    }
#pragma unroll
    for (int k = 0; k < WS - 1; ++k) {
      w0[k] = w0[k + 1];
      w1[k] = w1[k + 1];
      w2[k] = w2[k + 1];
    }
  }
  if constexpr (LAST) {
    if (a.partial) {
      for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
      const int w = threadIdx.x >> 6;
      if ((threadIdx.x & 63) == 0) red[w] = part;
      __syncthreads();
      if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int k = 0; k < kSfBlock / 64; ++k) sum += red[k];
        a.partial[(rhs * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = sum;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
int sumfac_bands(const HostProblem& hp, const double* V_quad, std::vector<double> out[3]) {
  const int d = hp.d, ps = hp.p_s, W = 2 * ps + 1;
  const double nu = hp.nu;
  int Q[3] = {1, 1, 1};
  size_t nq = 1;
  for (int l = 0; l < d; ++l) {
    Q[l] = int(hp.dir_s[l].x.size());
    nq *= size_t(Q[l]);
  }
  std::vector<double> v[3];
  for (int l = 0; l < d; ++l) v[l].assign(size_t(Q[l]), 0.0);
  if (V_quad) {
    // V = sum_l v_l(x_l): v_1(q) = V(q, 0, 0), v_l(q) = V(.., q, ..) - V(0, 0, 0) for l > 1; then every
    // sample must equal the sum (to rounding)
    size_t st[3] = {1, size_t(Q[0]), size_t(Q[0]) * size_t(Q[1])};
    for (int l = 0; l < d; ++l)
      for (int q = 0; q < Q[l]; ++q) v[l][size_t(q)] = V_quad[size_t(q) * st[l]] - (l > 0 ? V_quad[0] : 0.0);
    double vmax = 0.0;
    for (size_t k = 0; k < nq; ++k) {
      if (!std::isfinite(V_quad[k])) return 1;
      vmax = std::max(vmax, std::fabs(V_quad[k]));
    }
    for (size_t k = 0; k < nq; ++k) {
      size_t r = k;
      double s = 0.0;
      for (int l = 0; l < d; ++l) {
        s += v[l][r % size_t(Q[l])];
        r /= size_t(Q[l]);
      }
      if (std::fabs(V_quad[k] - s) > 1e-12 * vmax) return 1;
    }
  }
  for (int l = 0; l < d; ++l) {
    const Direction& D = hp.dir_s[l];
    const int n = hp.n_s[l];
    std::vector<double> Mv(size_t(n) * n, 0.0), Kv(size_t(n) * n, 0.0), Mv2(size_t(n) * n, 0.0);
    if (V_quad) {
      for (int e = 0; e < D.n_el; ++e)
        for (int g = 0; g < D.q; ++g) {
          const size_t qi = size_t(e) * D.q + g;
          const double w = D.w[qi], vv = v[l][qi];
          for (int a = 0; a <= D.p; ++a) {
            const int i = D.first[e] + a - 1;  // reduced index (first and last functions removed)
            if (i < 0 || i >= n) continue;
            const double bi = D.b(e, g, 0, a);
            for (int b = 0; b <= D.p; ++b) {
              const int j = D.first[e] + b - 1;
              if (j < 0 || j >= n) continue;
              const double bj = D.b(e, g, 0, b), bj2 = D.b(e, g, 2, b);
              Mv[size_t(i) * n + j] += w * vv * bi * bj;
              Kv[size_t(i) * n + j] += w * vv * bi * bj2;
              Mv2[size_t(i) * n + j] += w * vv * vv * bi * bj;
            }
          }
        }
    }
    out[l].assign(size_t(3) * n * W, 0.0);
    for (int i = 0; i < n; ++i)
      for (int o = 0; o < W; ++o) {
        const int j = i + o - ps;
        if (j < 0 || j >= n) continue;
        const size_t ij = size_t(i) * n + j, ji = size_t(j) * n + i;
        out[l][(size_t(0) * n + i) * W + o] = hp.Ms1[l][ij];
        out[l][(size_t(1) * n + i) * W + o] = nu * hp.Ls1[l][ij] + Mv[ij];
        out[l][(size_t(2) * n + i) * W + o] = nu * nu * hp.Js1[l][ij] - nu * (Kv[ij] + Kv[ji]) + Mv2[ij];
      }
  }
  return 0;
}

// rows per thread of an axis pass: segments of about kSfSeg rows, the same length for all
static int axis_segment(int n) {
  const int segs = std::max(1, (n + kSfSeg / 2) / kSfSeg);
  return std::min((n + segs - 1) / segs, kSfSegMax);
}

int sumfac_plan_shape(SumFacPlan& p, size_t max_lds) {
  if (p.d < 2 || p.d > 3 || p.ps < 2 || p.ps > 5 || p.pt < 1 || p.pt > 6) return -1;
  if (p.n_t > 128) return -1;  // one thread per time index, at most two waves
  const int n1 = p.n[0], nt = p.n_t;
  p.chunk = axis_segment(n1);
  const int W = 2 * p.ps + 1;
  p.lds = size_t(p.chunk + 2 * p.ps) * size_t(nt) * 16 + size_t(3) * p.chunk * W * sizeof(double);
  if (p.lds > std::min<size_t>(max_lds, 64 * 1024)) return -1;
  // axis passes: one thread per line and segment of about kSfSeg rows
  const int la = p.d - 1;
  p.seg_last = axis_segment(p.n[la]);
  if (p.seg_last > kSfSegMax || axis_segment(p.n[1]) > kSfSegMax) return -1;
  const int64_t lines_last = p.N / p.n[la];
  p.last_grid = int((lines_last + kSfBlock - 1) / kSfBlock) * ((p.n[la] + p.seg_last - 1) / p.seg_last);
  p.seg_mid = axis_segment(p.n[1]);
  return 0;
}

namespace {

template <int PS>
int launch_pass1_ps(const SumFacPlan& p, const SfPass1Args& a, dim3 grid, hipStream_t s) {
  switch (p.pt) {
#define STFD_SF1(PT)                                                                                        \
  case PT:                                                                                                  \
    hipLaunchKernelGGL((sf_pass1_kernel<PS, PT>), grid, dim3(p.n_t <= 64 ? 64 : 128), p.lds, s, a);        \
    break;
    STFD_SF1(1) STFD_SF1(2) STFD_SF1(3) STFD_SF1(4) STFD_SF1(5) STFD_SF1(6)
#undef STFD_SF1
    default:
      return -1;
  }
  return 0;
}

template <bool LAST>
int launch_axis(int ps, const SfAxisArgs& a, dim3 grid, hipStream_t s) {
  switch (ps) {
    case 2: hipLaunchKernelGGL((sf_axis_kernel<2, LAST>), grid, dim3(kSfBlock), 0, s, a); break;
    case 3: hipLaunchKernelGGL((sf_axis_kernel<3, LAST>), grid, dim3(kSfBlock), 0, s, a); break;
    case 4: hipLaunchKernelGGL((sf_axis_kernel<4, LAST>), grid, dim3(kSfBlock), 0, s, a); break;
    case 5: hipLaunchKernelGGL((sf_axis_kernel<5, LAST>), grid, dim3(kSfBlock), 0, s, a); break;
    default: return -1;
  }
  return 0;
}

}  // namespace

int sumfac_matvec(const SumFacPlan& p, const double* x, double* y, int64_t nrhs, double* partial, const int* done,
                  hipStream_t s) {
  if (nrhs < 1 || nrhs > 65535) return int(hipErrorInvalidValue);
  double2* w = reinterpret_cast<double2*>(p.work);
  const int64_t ws = p.work_stride / 2;
  double2* Z[3] = {w, w + ws, w + 2 * ws};
  SfPass1Args a1;
  a1.x = reinterpret_cast<const double2*>(x);
  a1.za = Z[0];
  a1.zb = Z[1];
  a1.zc = Z[2];
  a1.band = p.bands[0];
  a1.tband = p.tband;
  a1.n1 = p.n[0];
  a1.n_t = p.n_t;
  a1.seg = p.chunk;
  a1.segs = (p.n[0] + p.chunk - 1) / p.chunk;
  a1.N = p.N;
  a1.done = done;
  const int64_t pencils = p.N / (int64_t(p.n[0]) * p.n_t);
  const dim3 g1(unsigned(pencils * a1.segs), unsigned(nrhs));
  int rc = -1;
  switch (p.ps) {
    case 2: rc = launch_pass1_ps<2>(p, a1, g1, s); break;
    case 3: rc = launch_pass1_ps<3>(p, a1, g1, s); break;
    case 4: rc = launch_pass1_ps<4>(p, a1, g1, s); break;
    case 5: rc = launch_pass1_ps<5>(p, a1, g1, s); break;
    default: break;
  }
  if (rc) return int(hipErrorInvalidValue);
  const double2* last_in[3] = {Z[0], Z[1], Z[2]};
  if (p.d == 3) {
    double2* PQR[3] = {w + 3 * ws, w + 4 * ws, w + 5 * ws};
    SfAxisArgs am;
    for (int k = 0; k < 3; ++k) {
      am.in[k] = Z[k];
      am.out[k] = PQR[k];
      last_in[k] = PQR[k];
    }
    am.band = p.bands[1];
    am.n = p.n[1];
    am.seg = p.seg_mid;
    am.stride = int64_t(p.n_t) * p.n[0];
    am.lines = p.N / p.n[1];
    am.N = p.N;
    am.x = nullptr;
    am.partial = nullptr;
    am.done = done;
    const dim3 gm(unsigned((am.lines + kSfBlock - 1) / kSfBlock), unsigned((am.n + am.seg - 1) / am.seg),
                  unsigned(nrhs));
    if (launch_axis<false>(p.ps, am, gm, s)) return int(hipErrorInvalidValue);
  }
  SfAxisArgs al;
  for (int k = 0; k < 3; ++k) {
    al.in[k] = last_in[k];
    al.out[k] = nullptr;
  }
  al.out[0] = reinterpret_cast<double2*>(y);
  const int la = p.d - 1;
  al.band = p.bands[la];
  al.n = p.n[la];
  al.seg = p.seg_last;
  al.stride = int64_t(p.n_t) * p.n[0] * (la == 2 ? p.n[1] : 1);
  al.lines = p.N / p.n[la];
  al.N = p.N;
  al.x = reinterpret_cast<const double2*>(x);
  al.partial = partial;
  al.done = done;
  const dim3 gl(unsigned((al.lines + kSfBlock - 1) / kSfBlock), unsigned((al.n + al.seg - 1) / al.seg),
                unsigned(nrhs));
  if (launch_axis<true>(p.ps, al, gl, s)) return int(hipErrorInvalidValue);
  return int(hipGetLastError());
}

}  // namespace stfd
