// MI355X (gfx950) implementation of the C ABI in include/stfd.h.
//
// Hot path per PCG iteration (Section 5.3):
//   matvec  q = A p           : stencil x band kernel (FP64), fused <p,q> partials
//   update  x += a p, r -= a q: BLAS-1 with fused ||r||^2 partials
//   apply   z = P-hat^{-1} r  : 2d MFMA mode products + one banded time-solve kernel
//                                (Algorithm 1 steps 2-4)
//   dots / p-update           : Polak-Ribiere beta, p = z + beta p
// Reductions are deterministic: every block writes one partial per reduction
// and consumers sum the partials in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <type_traits>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/stfd.h"
#include "host_setup.h"
#include "kernels.h"
#include "load_vector.h"
#include "spatial.h"
#include "spatial_dev.h"
#include "sumfac.h"

namespace stfd {

#ifdef STFD_PHASE_TIMING
__device__ unsigned long long g_phase[4096][8];
__device__ unsigned long long g_cycles[4096][8];
#define STFD_STAMP(slot, k)                                                           \
  do {                                                                                \
    if (threadIdx.x == 0 && blockIdx.x < 4096) {                                      \
      g_phase[blockIdx.x][k] = __builtin_amdgcn_s_memrealtime();                      \
      g_cycles[blockIdx.x][k] = __builtin_amdgcn_s_memtime();                         \
    }                                                                                 \
  } while (0)
#else
#define STFD_STAMP(slot, k) \
  do {                      \
  } while (0)
#endif

static thread_local int g_last_hip_error = 0;

constexpr int kLag = 3;  // iterations the host lets the device run ahead of its convergence check

#define STFD_HIP(expr)                          \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) {                     \
      g_last_hip_error = int(e_);               \
      return STFD_EHIP;                         \
    }                                           \
  } while (0)

constexpr int kXcds = 8;  // MI355X: 8 accelerator complex dies, each with its own L2

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ short f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return short(u >> 16);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Ends a batch of loads: the compiler may neither sink a load of the batch below this point
// (into a branch that needs an earlier result, which would serialise the round trips) nor
// schedule arithmetic on its results between the loads.  Emits no instruction.
__device__ __forceinline__ void load_batch_end() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

// Deterministic block sum (fixed tree order); result valid in all threads.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < NT / 64; ++i) s += sh[i];
  return s;
}

// Sum of nparts partials (fixed order per thread, then block tree); all threads get it.  The loads
// of a thread are issued in batches of kSumBatch before any is added (one memory round trip per
// batch instead of one per partial).
constexpr int kSumBatch = 8;
template <int NT>
__device__ __forceinline__ double sum_partials(const double* parts, int nparts, double* sh) {
  double s = 0.0;
  for (int b0 = 0; b0 < nparts; b0 += NT * kSumBatch) {
    double v[kSumBatch];
#pragma unroll
    for (int u = 0; u < kSumBatch; ++u) {
      const int idx = b0 + u * NT + int(threadIdx.x);
      v[u] = idx < nparts ? parts[idx] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kSumBatch; ++u) s += v[u];
  }
  return block_sum<NT>(s, sh);
}

// Three sums of partials in one pass (a: na partials, b and c: nbc partials each).
template <int NT>
__device__ __forceinline__ void sum_partials3(const double* a, int na, const double* b, const double* c, int nbc,
                                              double* sh, double& sa, double& sb, double& sc) {
  double ta = 0.0, tb = 0.0, tc = 0.0;
  const int n = max(na, nbc);
  for (int b0 = 0; b0 < n; b0 += NT * kSumBatch) {
    double va[kSumBatch], vb[kSumBatch], vc[kSumBatch];
#pragma unroll
    for (int u = 0; u < kSumBatch; ++u) {
      const int idx = b0 + u * NT + int(threadIdx.x);
      va[u] = idx < na ? a[idx] : 0.0;
      vb[u] = idx < nbc ? b[idx] : 0.0;
      vc[u] = idx < nbc ? c[idx] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kSumBatch; ++u) {
      ta += va[u];
      tb += vb[u];
      tc += vc[u];
    }
  }
  sa = block_sum<NT>(ta, sh);
  sb = block_sum<NT>(tb, sh);
  sc = block_sum<NT>(tc, sh);
}

// ---------------------------------------------------------------------------
// Mode product (Algorithm 1 steps 2 and 4): Out[o][a][r] = sum_j U'[j][a] In[o][j][r].
// One wave = one group of 16 rows r of one outer slice o and one group of 16 output
// columns a; a block = kMpWaves waves on consecutive row tiles of one column group.
// The block stages the column group's U' fragments (packed at setup in the order the
// lanes read them) in LDS, and every wave loads the In fragments of its row group for
// all KS = ceil(n / K) K steps straight into registers in one batch, then runs one
// MFMA chain (U' from LDS) and the stores.  KS is exact per instantiation for FP64
// (padded K steps cost full MFMAs; a skipping branch breaks the load batch).  Block
// order: workgroups are dealt out round-robin over the XCDs, so logical block
// lb = (b % X)(grid / X) + b / X (the grid is a multiple of X) gives each XCD a
// contiguous range of (right-hand side, tile group, column group), column group
// fastest: the column groups of a tile, which read the same In fragments, and
// neighbouring tiles, whose 16-row fragments straddle the same cache lines when a row
// is not a multiple of 128 bytes, share one L2.  Tile groups are padded to a multiple
// of X per right-hand side; waves past the last tile only stage U' and write zero dot
// partials.  One dot partial pair per block, stored at the logical index.  The long
// directions keep one-wave blocks (one tile each) and read U' from global memory.
// MFMA computes C^T = U'^T A^T so that the 16 rows of a result fragment are
// contiguous in memory (coalesced stores).
//   FP64: v_mfma_f64_16x16x4f64, K step 4
//   FP32: v_mfma_f32_16x16x4f32, K step 4
//   BF16: v_mfma_f32_16x16x16bf16_1k, K step 16, FP32 accumulation
// Operand layouts (16x16xK, one block): lane l supplies A[m = l%16][k = (K/4)(l/16) + e]
// and B[k = (K/4)(l/16) + e][n = l%16].  Result register v of lane l holds
// D[m = 4(l/16) + v][n = l%16] for the FP32-accumulating instructions and
// D[m = 4v + l/16][n = l%16] for v_mfma_f64_16x16x4f64 (checked by the
// stfd_debug_mfma_layout probe).
// ---------------------------------------------------------------------------
template <int PREC>
struct MPTraits;
// u_t: storage type of the U' operand the kernel reads (an FP32 copy for the FP32 and BF16
// products: the value converted at use is the same, half the bytes)
template <>
struct MPTraits<MP_F64> {
  using op_t = double;
  using acc_t = d4_t;
  using u_t = double;
  static constexpr int K = 4;
};
template <>
struct MPTraits<MP_F32> {
  using op_t = float;
  using acc_t = f4_t;
  using u_t = float;
  static constexpr int K = 4;
};
template <>
struct MPTraits<MP_BF16> {
  using op_t = short;  // bf16 bits
  using acc_t = f4_t;
  using u_t = float;
  static constexpr int K = 16;
};

template <int PREC>
__device__ __forceinline__ typename MPTraits<PREC>::op_t to_op(double v) {
  if constexpr (PREC == MP_F64) return v;
  else if constexpr (PREC == MP_F32) return float(v);
  else return f32_to_bf16(float(v));
}
template <int PREC>
__device__ __forceinline__ typename MPTraits<PREC>::op_t to_op(float v) {
  if constexpr (PREC == MP_F64) return double(v);
  else if constexpr (PREC == MP_F32) return v;
  else return f32_to_bf16(v);
}

// Remainder columns.  Where n = 16 g + r with g >= 1 and r <= 2, the last r output columns would
// take a 16-column MFMA group of their own, at least 14/16 of it padding (n = 65 in 2D and 49 in
// 3D at p = 3: 20 and 25% of the MFMA work and of the narrow form's waves).  Instead they are
// computed with vector FMAs from the In values the wave already holds: a lane sums
// U'[j][a] In[j][row] over its own K rows j = ks K + E grp + e in K-step order, and two butterfly
// rounds over the four lane groups complete the sum in every lane.  FP64 and FP32 products only
// (operands rounded as the MFMA rounds them, summed in its accumulator type); BF16 keeps the MFMA
// group.  The narrow and the wide form run this same sequence, so they still agree bit for bit.
template <int PREC>
using rem_acc_t = typename std::conditional<PREC == MP_F64, double, float>::type;
template <int PREC, typename U, typename X>
__device__ __forceinline__ rem_acc_t<PREC> rem_step(U u, X x, bool in_k, rem_acc_t<PREC> s) {
  static_assert(PREC != MP_BF16, "no remainder columns in BF16 products");
  if constexpr (PREC == MP_F64) {
    return __builtin_fma(double(u), in_k ? double(x) : 0.0, s);
  } else {
    return __builtin_fmaf(float(u), in_k ? float(x) : 0.0f, s);
  }
}
template <typename A>
__device__ __forceinline__ A rem_finish(A s) {
  s += __shfl_xor(s, 16, 64);
  s += __shfl_xor(s, 32, 64);
  return s;
}

// Row tiles per block of the one-group form: the waves of a block take consecutive row tiles of one
// column group, so the block stages that group's packed U' in LDS once and every wave reads its
// fragments there instead of from global memory (half of the form's vector memory instructions).
constexpr int kMpWaves = 4;
template <int PREC, typename Tin, typename Tout, int KS, int RT, bool DOT, int RC, bool LDSU>
__global__ __launch_bounds__(64 * kMpWaves) void mode_product_kernel(ModeProductArgs a) {
  using Tr = MPTraits<PREC>;
  using op_t = typename Tr::op_t;
  using u_t = typename Tr::u_t;
  constexpr int K = Tr::K;
  constexpr int E = K / 4;
  constexpr int NT = 64 * kMpWaves;
  constexpr int UG = KS * 64 * E;                             // packed U' values of one column group
  constexpr int US = LDSU ? (RC > 0 ? 2 : 1) * UG : 1;        // staged: the group (and the remainder's)
  constexpr int UPT = LDSU ? (US + NT - 1) / NT : 1;          // staged values per thread
  __shared__ u_t Us[US];
  __shared__ double red[2][kMpWaves];
  const int n = a.n;
  const int64_t per_rhs = int64_t(a.groups) * a.tiles_pad;
  const int64_t lb = int64_t(blockIdx.x % kXcds) * (gridDim.x / kXcds) + blockIdx.x / kXcds;
  const int64_t rhs = lb / per_rhs;
  if (a.done && a.done[rhs]) return;  // uniform per block
  STFD_STAMP(1, 4);
  const int64_t remb = lb - rhs * per_rhs;
  const int64_t tgrp = remb / a.groups;
  const int cg = int(remb - tgrp * a.groups);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t tile = tgrp * kMpWaves + wave;
  const bool active = tile < a.tiles_per_rhs;
  // remainder columns 16 groups + c, c < RC, computed by the waves of the last MFMA group; their
  // U' values are the packed group after the last MFMA group
  const bool rem_wave = RC > 0 && cg == a.groups - 1;
  // staging loads first: waiting for them before the LDS writes then leaves the In loads in flight
  u_t stg[UPT];
  if constexpr (LDSU) {
    const u_t* Ug = static_cast<const u_t*>(a.U) + int64_t(cg) * UG;
    const int cnt = rem_wave ? US : UG;
#pragma unroll
    for (int u = 0; u < UPT; ++u) {
      const int i = u * NT + int(threadIdx.x);
      stg[u] = i < cnt ? Ug[i] : u_t(0);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  double dot_a = 0.0, dot_b = 0.0;
  // a tile is RT adjacent 16-row groups: one U' fragment serves RT MFMA chains and a row of In is
  // read as 16 RT consecutive values
  const int64_t ti = active ? tile : 0;
  const int64_t o = rhs * a.outer_per_rhs + ti / a.n_row_tiles;
  const int64_t row0 = (ti % a.n_row_tiles) * (16 * RT);
  const int rows_here = int(min<int64_t>(16 * RT, a.inner - row0));
  const Tin* src = static_cast<const Tin*>(a.in) + o * int64_t(n) * a.inner + row0;
  Tout* dst = static_cast<Tout*>(a.out) + o * int64_t(n) * a.inner + row0;
  const int a0 = cg * 16;
  const int col = lane & 15, grp = lane >> 4;
  // operand fragments: A = U'^T (m = column a0 + col), B = In (n = row 16 t + col), k = j; In
  // addresses are clamped into the operand and values past n replaced by zeros
  int rc[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) rc[t] = min(16 * t + col, rows_here - 1);
  // without LDS staging (one operand per outer slice): this lane's U' values from global memory
  // (packed in fragment order, see pack_mode_operand; zero past n)
  const u_t* Up = static_cast<const u_t*>(a.U) + (a.u_slice_stride ? (o % a.outer_per_rhs) * a.u_slice_stride : 0) +
                  int64_t(cg) * UG + lane * E;
  u_t ur[LDSU ? 1 : KS][E];
  u_t urm[(RC > 0 && !LDSU) ? RC : 1][LDSU ? 1 : KS][E];
  double rrm[RT][RC > 0 ? RC : 1], zrm[RT][RC > 0 ? RC : 1];
  if constexpr (RC > 0 && !LDSU) {
    if (rem_wave) {
      const u_t* Ur = Up - lane * E + UG + grp * 16 * E;
#pragma unroll
      for (int c = 0; c < RC; ++c)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
          for (int e = 0; e < E; ++e) urm[c][ks][e] = Ur[(ks * 64 + c) * E + e];
    }
  }
  if constexpr (RC > 0 && DOT) {
    if (rem_wave) {
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int c = 0; c < RC; ++c) {
          const int64_t g = o * int64_t(n) * a.inner + row0 + int64_t(16 * a.groups + c) * a.inner + rc[t];
          rrm[t][c] = a.dot_r[g];
          zrm[t][c] = a.dot_z[g];
        }
    }
  }
  Tin xr[RT][KS][E];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int jc = min(ks * K + E * grp + e, n - 1);
      if constexpr (!LDSU) ur[ks][e] = Up[ks * 64 * E + e];
#pragma unroll
      for (int t = 0; t < RT; ++t) xr[t][ks][e] = src[int64_t(jc) * a.inner + rc[t]];
    }
  // operands of the fused dot products (last backward product of a PCG iteration; a template
  // switch, so that no branch separates these loads from the operand loads)
  double rv[RT][4], zv[RT][4];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if constexpr (DOT) {
        const int aa = min(a0 + (PREC == MP_F64 ? 4 * v + grp : 4 * grp + v), n - 1);
        const int64_t g = o * int64_t(n) * a.inner + row0 + int64_t(aa) * a.inner + rc[t];
        rv[t][v] = a.dot_r[g];
        zv[t][v] = a.dot_z[g];
      } else {
        rv[t][v] = 0.0;
        zv[t][v] = 0.0;
      }
    }
  // keep every load above the MFMA chains (the scheduler would otherwise interleave them to save
  // registers, turning one memory latency into several); masking and conversion happen below
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (LDSU) {
#pragma unroll
    for (int u = 0; u < UPT; ++u) {
      const int i = u * NT + int(threadIdx.x);
      if (i < US) Us[i] = stg[u];
    }
    __syncthreads();
  }
  STFD_STAMP(1, 5);
  if (active) {
    typename Tr::acc_t acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[t] = typename Tr::acc_t{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      op_t ua[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if constexpr (LDSU) ua[e] = to_op<PREC>(Us[(ks * 64 + lane) * E + e]);
        else ua[e] = to_op<PREC>(ur[ks][e]);
      }
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        op_t xb[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const bool in_k = ks * K + E * grp + e < n;
          xb[e] = to_op<PREC>(in_k ? xr[t][ks][e] : Tin(0));
        }
        if constexpr (PREC == MP_F64) {
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ua[0], xb[0], acc[t], 0, 0, 0);
        } else if constexpr (PREC == MP_F32) {
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ua[0], xb[0], acc[t], 0, 0, 0);
        } else {
          s4_t av, bv;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            av[e] = ua[e];
            bv[e] = xb[e];
          }
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[t], 0, 0, 0);
        }
      }
    }
    STFD_STAMP(1, 6);
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      if (16 * t + col < rows_here) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int aa = a0 + (PREC == MP_F64 ? 4 * v + grp : 4 * grp + v);
          if (aa < n) {
            const int64_t off = int64_t(aa) * a.inner + 16 * t + col;
            dst[off] = Tout(acc[t][v]);
            if constexpr (DOT) {
              dot_a += rv[t][v] * double(Tout(acc[t][v]));
              dot_b += rv[t][v] * zv[t][v];
            }
          }
        }
      }
    }
    if constexpr (RC > 0) {
      if (rem_wave) {
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int c = 0; c < RC; ++c) {
            rem_acc_t<PREC> sum = 0;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
              for (int e = 0; e < E; ++e) {
                u_t um;
                if constexpr (LDSU) um = Us[UG + (ks * 64 + grp * 16 + c) * E + e];
                else um = urm[c][ks][e];
                sum = rem_step<PREC>(um, xr[t][ks][e], ks * K + E * grp + e < n, sum);
              }
            sum = rem_finish(sum);
            if (grp == 0 && 16 * t + col < rows_here) {
              const Tout val = Tout(sum);
              dst[int64_t(16 * a.groups + c) * a.inner + 16 * t + col] = val;
              if constexpr (DOT) {
                dot_a += rrm[t][c] * double(val);
                dot_b += rrm[t][c] * zrm[t][c];
              }
            }
          }
      }
    }
  }
  if constexpr (DOT) {
    // one partial pair per block, stored at the logical block index (waves in order)
    dot_a = wave_sum(dot_a);
    dot_b = wave_sum(dot_b);
    if (lane == 0) {
      red[0][wave] = dot_a;
      red[1][wave] = dot_b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double sa = 0.0, sb = 0.0;
#pragma unroll
      for (int w = 0; w < kMpWaves; ++w) {
        sa += red[0][w];
        sb += red[1][w];
      }
      a.part_a[lb] = sa;
      a.part_b[lb] = sb;
    }
  }
  STFD_STAMP(1, 7);
}

// ---------------------------------------------------------------------------
// Mode product for long directions (n > kMaxModeN, one spatial direction): the one-group form
// with one 16-row group per wave and the K steps walked in chunks of kLongChunk (each chunk's
// operand loads in one batch, then its MFMA chain), so the register footprint does not grow with
// n.  One wave per block (one row tile) and U' read from global memory; K-step order and
// epilogue as in mode_product_kernel.
// ---------------------------------------------------------------------------
constexpr int kLongChunk = 16;

template <int PREC, typename Tin, typename Tout, bool DOT>
__global__ __launch_bounds__(64) void mode_product_long_kernel(ModeProductArgs a, int KS) {
  using Tr = MPTraits<PREC>;
  using op_t = typename Tr::op_t;
  using u_t = typename Tr::u_t;
  constexpr int K = Tr::K;
  constexpr int E = K / 4;
  const int n = a.n;
  const int64_t per_rhs = int64_t(a.groups) * a.tiles_pad;
  const int64_t lb = int64_t(blockIdx.x % kXcds) * (gridDim.x / kXcds) + blockIdx.x / kXcds;
  const int64_t rhs = lb / per_rhs;
  if (a.done && a.done[rhs]) return;
  const int64_t rem = lb - rhs * per_rhs;
  const int64_t tile = rem / a.groups;
  const int cg = int(rem - tile * a.groups);
  const int lane = threadIdx.x;
  double dot_a = 0.0, dot_b = 0.0;
  if (tile < a.tiles_per_rhs) {
    const int64_t o = rhs * a.outer_per_rhs + tile / a.n_row_tiles;
    const int64_t row0 = (tile % a.n_row_tiles) * 16;
    const int rows_here = int(min<int64_t>(16, a.inner - row0));
    const Tin* src = static_cast<const Tin*>(a.in) + o * int64_t(n) * a.inner + row0;
    Tout* dst = static_cast<Tout*>(a.out) + o * int64_t(n) * a.inner + row0;
    const int a0 = cg * 16;
    const int col = lane & 15, grp = lane >> 4;
    const int rc = min(col, rows_here - 1);
    const u_t* Up = static_cast<const u_t*>(a.U) + (int64_t(cg) * KS * 64 + lane) * E;
    typename Tr::acc_t acc = typename Tr::acc_t{0, 0, 0, 0};
    for (int k0 = 0; k0 < KS; k0 += kLongChunk) {
      u_t ur[kLongChunk][E];
      Tin xr[kLongChunk][E];
#pragma unroll
      for (int c = 0; c < kLongChunk; ++c) {
        const int kc = min(k0 + c, KS - 1);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int jc = min(kc * K + E * grp + e, n - 1);
          ur[c][e] = Up[int64_t(kc) * 64 * E + e];
          xr[c][e] = src[int64_t(jc) * a.inner + rc];
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int c = 0; c < kLongChunk; ++c) {
        if (k0 + c < KS) {  // uniform
          op_t ua[E], xb[E];
#pragma unroll
          for (int e = 0; e < E; ++e) {
            ua[e] = to_op<PREC>(ur[c][e]);
            xb[e] = to_op<PREC>((k0 + c) * K + E * grp + e < n ? xr[c][e] : Tin(0));
          }
          if constexpr (PREC == MP_F64) {
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ua[0], xb[0], acc, 0, 0, 0);
          } else if constexpr (PREC == MP_F32) {
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ua[0], xb[0], acc, 0, 0, 0);
          } else {
            s4_t av, bv;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              av[e] = ua[e];
              bv[e] = xb[e];
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
          }
        }
      }
    }
    if (col < rows_here) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int aa = a0 + (PREC == MP_F64 ? 4 * v + grp : 4 * grp + v);
        if (aa < n) {
          const int64_t off = int64_t(aa) * a.inner + col;
          const Tout val = Tout(acc[v]);
          dst[off] = val;
          if constexpr (DOT) {
            const int64_t g = o * int64_t(n) * a.inner + row0 + off;
            const double rv = a.dot_r[g];
            dot_a += rv * double(val);
            dot_b += rv * a.dot_z[g];
          }
        }
      }
    }
  }
  if constexpr (DOT) {
    dot_a = wave_sum(dot_a);
    dot_b = wave_sum(dot_b);
    if (lane == 0) {
      a.part_a[lb] = dot_a;
      a.part_b[lb] = dot_b;
    }
  }
}

// ---------------------------------------------------------------------------
// Mode product, wide form (large launches with one operand): a wave computes all G = ceil(n / 16)
// column groups of a 16-row tile, so every In fragment it loads feeds G MFMA chains instead of one,
// and the packed operand U' of all groups is staged in LDS once per block of 4 waves.  A block
// walks the tiles of its right-hand side in rounds of 4 consecutive tiles (which share the cache
// lines straddling their boundaries) with a stride of 4 blocks_per_rhs tiles.  Per tile the vector
// memory pipeline moves 1/G of the In bytes and none of the U' bytes of the one-group form.
// Grid (blocks_per_rhs, nrhs); the fused dot products write one partial pair per block.
// ---------------------------------------------------------------------------
// Waves per SIMD asked of the compiler: the grid is kMpWideBlocks blocks of 4 waves, so 4 blocks
// per CU hold it in one round; with 3 the last quarter of the blocks runs alone after the rest
// (3D p = 3 48^4, n = 49: 41 us per product at 3 waves).  Asked only where the compiler's resource
// report shows 4 waves (128 registers, accumulators in VGPRs) without spilling; elsewhere its own
// choice stands.
template <int PREC, int KS, bool DOT, int RC>
constexpr int mode_product_wide_waves() {
  return (PREC == MP_F64 && !DOT && (KS <= 10 || (KS == 12 && RC == 0) || (KS == 13 && RC == 1))) ? 4 : 1;
}
template <int PREC, typename Tin, typename Tout, int KS, bool DOT, int RC>
__global__ __launch_bounds__(256, (mode_product_wide_waves<PREC, KS, DOT, RC>())) void mode_product_wide_kernel(
    ModeProductArgs a, int64_t blocks_per_rhs) {
  using Tr = MPTraits<PREC>;
  using op_t = typename Tr::op_t;
  using u_t = typename Tr::u_t;
  constexpr int K = Tr::K;
  constexpr int E = K / 4;
  constexpr int G = PREC == MP_BF16 ? KS : (KS + 3) / 4;  // column groups of the packed operand
  constexpr int GM = RC > 0 ? G - 1 : G;                   // of them computed by MFMA chains
  __shared__ u_t Us[G * KS * 64 * E];
  __shared__ double red[2][4];
  const int64_t rhs = blockIdx.y;
  if (a.done && a.done[rhs]) return;  // uniform per block
  const u_t* Ug = static_cast<const u_t*>(a.U);
  for (int i = threadIdx.x; i < G * KS * 64 * E; i += blockDim.x) Us[i] = Ug[i];
  __syncthreads();
  const int n = a.n;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  double dot_a = 0.0, dot_b = 0.0;
  for (int64_t t0 = int64_t(blockIdx.x) * 4; t0 < a.tiles_per_rhs; t0 += blocks_per_rhs * 4) {
    const int64_t tile = t0 + wave;
    if (tile >= a.tiles_per_rhs) break;
    const int64_t o = rhs * a.outer_per_rhs + tile / a.n_row_tiles;
    const int64_t row0 = (tile % a.n_row_tiles) * 16;
    const int rows_here = int(min<int64_t>(16, a.inner - row0));
    const int64_t base = o * int64_t(n) * a.inner + row0;
    const Tin* src = static_cast<const Tin*>(a.in) + base;
    Tout* dst = static_cast<Tout*>(a.out) + base;
    const int rc = min(col, rows_here - 1);
    Tin xr[KS][E];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int e = 0; e < E; ++e) xr[ks][e] = src[int64_t(min(ks * K + E * grp + e, n - 1)) * a.inner + rc];
    // operands of the fused dot products, in the same batch as In (loaded after the stores they
    // would wait behind every store: the compiler cannot tell that r, z_old and Out do not overlap)
    double rv[DOT ? GM : 1][4], zv[DOT ? GM : 1][4];
    double rrm[RC > 0 ? RC : 1], zrm[RC > 0 ? RC : 1];
    if constexpr (DOT) {
#pragma unroll
      for (int g = 0; g < GM; ++g)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int aa = min(16 * g + (PREC == MP_F64 ? 4 * v + grp : 4 * grp + v), n - 1);
          const int64_t off = base + int64_t(aa) * a.inner + rc;
          rv[g][v] = a.dot_r[off];
          zv[g][v] = a.dot_z[off];
        }
#pragma unroll
      for (int c = 0; c < RC; ++c) {
        const int64_t off = base + int64_t(16 * GM + c) * a.inner + rc;
        rrm[c] = a.dot_r[off];
        zrm[c] = a.dot_z[off];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    typename Tr::acc_t acc[GM];
#pragma unroll
    for (int g = 0; g < GM; ++g) acc[g] = typename Tr::acc_t{0, 0, 0, 0};
    rem_acc_t<PREC> rsum[RC > 0 ? RC : 1];
#pragma unroll
    for (int c = 0; c < RC; ++c) rsum[c] = 0;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      op_t xb[E];
#pragma unroll
      for (int e = 0; e < E; ++e) xb[e] = to_op<PREC>(ks * K + E * grp + e < n ? xr[ks][e] : Tin(0));
#pragma unroll
      for (int g = 0; g < GM; ++g) {
        op_t ua[E];
#pragma unroll
        for (int e = 0; e < E; ++e) ua[e] = to_op<PREC>(Us[((g * KS + ks) * 64 + lane) * E + e]);
        if constexpr (PREC == MP_F64) {
          acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(ua[0], xb[0], acc[g], 0, 0, 0);
        } else if constexpr (PREC == MP_F32) {
          acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(ua[0], xb[0], acc[g], 0, 0, 0);
        } else {
          s4_t av, bv;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            av[e] = ua[e];
            bv[e] = xb[e];
          }
          acc[g] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[g], 0, 0, 0);
        }
      }
      // remainder columns 16 GM + c: vector FMAs beside the MFMA chains (U' of packed group GM,
      // lane grp * 16 + c, an LDS broadcast)
      if constexpr (RC > 0) {
#pragma unroll
        for (int c = 0; c < RC; ++c)
#pragma unroll
          for (int e = 0; e < E; ++e)
            rsum[c] = rem_step<PREC>(Us[((GM * KS + ks) * 64 + grp * 16 + c) * E + e], xr[ks][e],
                                     ks * K + E * grp + e < n, rsum[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < RC; ++c) rsum[c] = rem_finish(rsum[c]);
    if (col < rows_here) {
#pragma unroll
      for (int g = 0; g < GM; ++g)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int aa = 16 * g + (PREC == MP_F64 ? 4 * v + grp : 4 * grp + v);
          if (aa < n) {
            const int64_t off = int64_t(aa) * a.inner + col;
            const Tout val = Tout(acc[g][v]);
            dst[off] = val;
            if constexpr (DOT) {
              dot_a += rv[DOT ? g : 0][v] * double(val);
              dot_b += rv[DOT ? g : 0][v] * zv[DOT ? g : 0][v];
            }
          }
        }
      if (grp == 0) {
#pragma unroll
        for (int c = 0; c < RC; ++c) {
          const Tout val = Tout(rsum[c]);
          dst[int64_t(16 * GM + c) * a.inner + col] = val;
          if constexpr (DOT) {
            dot_a += rrm[c] * double(val);
            dot_b += rrm[c] * zrm[c];
          }
        }
      }
    }
  }
  if constexpr (DOT) {
    dot_a = wave_sum(dot_a);
    dot_b = wave_sum(dot_b);
    if (lane == 0) {
      red[0][wave] = dot_a;
      red[1][wave] = dot_b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      a.part_a[rhs * blocks_per_rhs + blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
      a.part_b[rhs * blocks_per_rhs + blockIdx.x] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
  }
}

// ---------------------------------------------------------------------------
// Banded time solves (Algorithm 1 step 3): for every spatial mode i solve
// H_i x_i = y_i, H_i = L_t + mu_i^2 M_t + i mu_i K_t (Section 5.2), Hermitian
// positive definite with half-bandwidth P, factorised at setup as L D L^H
// (unit lower band L, real D > 0).
// A single sweep over n_t rows is a chain of 2 n_t dependent steps, and with one
// lane per mode the grid holds only N_s lanes.  Here each mode's rows are cut
// into S segments of LEN rows (the last padded with zero rows) and lane
// m*S + s of a 64-lane block keeps segment s of mode m in registers (rows of y,
// L and 1/D).  The forward substitution z = L^{-1} y is exact in three steps:
//  (1) sweep the segment from a zero history; its last P values are the local
//      tail;
//  (2) reduced recurrence tail_s = tail~_s + Tf_s tail_{s-1} over the segments,
//      S-1 rounds of neighbour-lane shuffles (Tf_s = P x P response of the
//      segment's last P values to its history, computed by the lane from its rows
//      of L: P homogeneous sweeps that do not depend on y, so they overlap the
//      sweep of step 1 and nothing but L and 1/D is read per row);
//  (3) sweep again from the true history tail_{s-1}; w = z / D.
// The backward substitution x = L^{-H} w takes the same three steps from the
// other end (future = first P values of the next segment, transfer Tb_s).
// Dependent chain per lane: 4 LEN sweep steps + 2 (S-1) reduced steps.
// FP64 applies solve in FP64; the FP32 and BF16 applies store y in FP32 and solve in FP32 with
// FP32 copies of the tables (half the table traffic).
// Table layouts: time_solve_plan in host_setup.h.
// ---------------------------------------------------------------------------
constexpr int kTsLanes = 64;
// compiled (P, LEN) pairs; the segment lengths offered per P by time_segment_length
#define STFD_TS_INSTANCES                                                                                    \
  STFD_TS(1, 8) STFD_TS(1, 16) STFD_TS(2, 8) STFD_TS(2, 12) STFD_TS(2, 16) STFD_TS(3, 6) STFD_TS(3, 8)       \
  STFD_TS(3, 12)                                                                                               \
  STFD_TS(3, 16) STFD_TS(4, 6) STFD_TS(4, 8) STFD_TS(4, 12) STFD_TS(5, 6) STFD_TS(5, 8) STFD_TS(6, 6)

// complex pair of the table / arithmetic type A
template <typename A>
struct TsVec;
template <>
struct TsVec<double> {
  using t = double2;
};
template <>
struct TsVec<float> {
  using t = float2;
};

// T: storage type of y; A: arithmetic and table type (double for FP64 solves, float for the FP32
// time solves of the mixed-precision applies, whose tables are FP32 copies of the FP64 ones)
// MODE 0: rows of L, 1/D and the transfers Tf, Tb read from tables (small grids: at most one wave
// per SIMD, bound by the dependent chain, which computing them would lengthen);
// MODE 1: rows of L and 1/D from tables, transfers computed in the solve;
// MODE 2: transfers computed and the rows of L and 1/D factorised in the solve from the segment's
// entry state Sf (the last P rows of the factor before the segment) and the time bands Hb (large
// grids: the kernel is bound by table traffic, and the state is P^2 values per segment instead of
// LEN (2P + 1)).  The row recurrence is the banded LDL^H step of the host factorisation:
//   L[t][t-k] = (H[t][t-k] - sum_{kk > k} L[t][t-kk] D[t-kk] conj(L[t-k][t-kk])) / D[t-k],
//   D[t] = Re H[t][t] - sum_k |L[t][t-k]|^2 D[t-k].
// 1 / x from the hardware reciprocal refined by Newton steps (two in FP64, one in FP32): within
// an ulp of the quotient, without the scaling and fix-up sequence of an IEEE division (x > 0 and
// normal here: the pivots of a Hermitian positive definite matrix)
__device__ __forceinline__ double ts_recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float ts_recip(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}

template <int MODE>
struct TsMode {
  static constexpr bool kFlyTransfers = MODE >= 1;
  static constexpr bool kFactor = MODE == 2;
};

// One lane of the segmented solve: segment s of one mode, whose n_t rows start at yb (global or
// LDS memory).  tl: the lane's slot in the table layout (rows of L, 1/D, transfers, entry states;
// tl + 1 holds the next segment of the same mode); pl: the lane in its wave (shuffles exchange
// with pl +- 1, which must hold the neighbouring segments of the same mode, and the parking slots
// Tsh / Dsh of the wave are indexed by it).  Table pointers are offset to the lane's table block.
template <typename T, typename A>
struct TsLaneArgs {
  typename TsVec<T>::t* yb;
  bool live;
  int s, segs, n_t;
  int tl, pl;
  const A* Lf;
  const A* Df;
  const A* Tf;
  const A* Tb;
  const A* Sf;
  const A* Hb;
  A mu;
  typename TsVec<A>::t* Tsh;  // [P * P][64] of the wave
  A* Dsh;                     // [LEN][64] of the wave (factor form)
};

template <typename T, typename A, int P, int LEN, int MODE>
__device__ __forceinline__ void time_solve_lane(const TsLaneArgs<T, A>& g) {
  constexpr bool FLY = TsMode<MODE>::kFlyTransfers;
  constexpr bool FACTOR = TsMode<MODE>::kFactor;
  using A2 = typename TsVec<A>::t;
  using T2 = typename TsVec<T>::t;
  const int s = g.s, segs = g.segs, n_t = g.n_t;
  const bool live = g.live;
  const int lane = g.tl;
  const int t0 = s * LEN;
  T2* yb = g.yb;
  const A2* Lb = reinterpret_cast<const A2*>(g.Lf);
  const A* Db = g.Df;
  A2* Tsh = g.Tsh;
  A* Dsh = g.Dsh;
  const A2* Tfb = reinterpret_cast<const A2*>(g.Tf);
  const A2* Tbb = reinterpret_cast<const A2*>(g.Tb);
  const A* Hb = g.Hb;

  // rows of y loaded (clamped addresses) and converted after the whole batch (the compiler moves a
  // conversion next to its load, which made every row wait for its own round trip); rows past n_t
  // and idle lanes are masked at the conversion
  A yr[LEN], yi[LEN], lr[LEN][P], li[LEN][P];
  T2 yv[LEN];
  // the inverse pivots of the table forms are loaded where they are used (with the rows above, the
  // extra registers spilled into AGPR copies inside the dependent sweeps)
  A tfr[P][P], tfi[P][P], tbr[P][P], tbi[P][P], dv[LEN];
  const bool has_next = s + 1 < segs;
  const int nxt = min(lane + 1, kTsLanes - 1);
  A nlr[P][P], nli[P][P];
  if constexpr (!FACTOR) {
#pragma unroll
    for (int j = 0; j < LEN; ++j) {
#pragma unroll
      for (int k = 0; k < P; ++k) {
        const A2 v = Lb[(j * P + k) * kTsLanes + lane];
        lr[j][k] = v.x;
        li[j][k] = v.y;
      }
      yv[j] = yb[min(t0 + j, n_t - 1)];
    }
    // L[t+k][t] for rows t+k of the next segment (rows jj < P of the neighbour lane)
#pragma unroll
    for (int jj = 0; jj < P; ++jj)
#pragma unroll
      for (int k = 0; k < P; ++k) {
        nlr[jj][k] = nli[jj][k] = A(0);
        if (k >= jj) {
          const A2 v = Lb[(jj * P + k) * kTsLanes + nxt];
          nlr[jj][k] = has_next ? v.x : A(0);
          nli[jj][k] = has_next ? v.y : A(0);
        }
      }
  } else {
    // entry state: window row a - 1 = row t0 - a (a = 1..P) with its entries L[t0-a][t0-a-k]
    // (k = 1..P-a) and D[t0-a], 1/D[t0-a]
    A wr[P][P], wi[P][P], wd[P], wdi[P];
    const A* Sb = g.Sf + lane;
    const A mu = g.mu;
    {
      int q = 0;
#pragma unroll
      for (int a = 1; a <= P; ++a)
#pragma unroll
        for (int k = 1; k <= P; ++k) {
          wr[a - 1][k - 1] = wi[a - 1][k - 1] = A(0);
          if (k <= P - a) {
            wr[a - 1][k - 1] = Sb[(q++) * kTsLanes];
            wi[a - 1][k - 1] = Sb[(q++) * kTsLanes];
          }
        }
#pragma unroll
      for (int a = 1; a <= P; ++a) {
        wd[a - 1] = Sb[(q++) * kTsLanes];
        wdi[a - 1] = ts_recip(wd[a - 1]);
      }
    }
    const A mu2 = mu * mu;
#pragma unroll
    for (int j = 0; j < LEN; ++j) {
      const int t = t0 + j;
      const A* hb = Hb + int64_t(t) * ((P + 1) * 3);  // padded rows carry zeros
      A nr[P + 1], ni[P + 1];  // nr[k] + i ni[k] = L[t][t-k]
#pragma unroll
      for (int k = P; k >= 1; --k) {
        // H[t][t-k] = L_t + mu^2 M_t + i mu K_t
        A sr = fma(mu2, hb[k * 3 + 1], hb[k * 3]);
        A si = mu * hb[k * 3 + 2];
#pragma unroll
        for (int kk = k + 1; kk <= P; ++kk) {
          // L[t][t-kk] D[t-kk] conj(L[t-k][t-kk]); row t-k is window row k-1, entry kk-k
          const A pr = nr[kk] * wd[kk - 1], pi = ni[kk] * wd[kk - 1];
          const A cr = wr[k - 1][kk - k - 1], ci = wi[k - 1][kk - k - 1];
          sr -= fma(pr, cr, pi * ci);
          si -= fma(pi, cr, -pr * ci);
        }
        nr[k] = sr * wdi[k - 1];
        ni[k] = si * wdi[k - 1];
      }
      A dt = fma(mu2, hb[1], hb[0]);
#pragma unroll
      for (int k = 1; k <= P; ++k) dt -= fma(nr[k], nr[k], ni[k] * ni[k]) * wd[k - 1];
      const bool row = t < n_t;
      const A dinv = row ? ts_recip(dt) : A(0);
#pragma unroll
      for (int k = 1; k <= P; ++k) {
        lr[j][k - 1] = row ? nr[k] : A(0);
        li[j][k - 1] = row ? ni[k] : A(0);
      }
      Dsh[j * kTsLanes + g.pl] = dinv;  // parked until step 3 (registers are the occupancy limit)
      // shift the window: row t becomes window row 0 with its entries k = 1..P-1
#pragma unroll
      for (int a = P - 1; a >= 1; --a) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
          wr[a][k] = wr[a - 1][k];
          wi[a][k] = wi[a - 1][k];
        }
        wd[a] = wd[a - 1];
        wdi[a] = wdi[a - 1];
      }
#pragma unroll
      for (int k = 1; k <= P; ++k) {
        wr[0][k - 1] = k < P ? nr[k] : A(0);
        wi[0][k - 1] = k < P ? ni[k] : A(0);
      }
      wd[0] = row ? dt : A(1);
      wdi[0] = row ? dinv : A(1);
    }
    // rows of y after the factorisation (its registers are free by then)
#pragma unroll
    for (int j = 0; j < LEN; ++j) yv[j] = yb[min(t0 + j, n_t - 1)];
    // L[t+k][t] of the next segment's first P rows, from the neighbour lane
#pragma unroll
    for (int jj = 0; jj < P; ++jj)
#pragma unroll
      for (int k = 0; k < P; ++k) {
        const A vr = __shfl_down(lr[jj < LEN ? jj : 0][k], 1), vi = __shfl_down(li[jj < LEN ? jj : 0][k], 1);
        nlr[jj][k] = (k >= jj && has_next) ? vr : A(0);
        nli[jj][k] = (k >= jj && has_next) ? vi : A(0);
      }
  }
  load_batch_end();
#pragma unroll
  for (int j = 0; j < LEN; ++j) {
    const bool ok = live && t0 + j < n_t;
    yr[j] = ok ? A(yv[j].x) : A(0);
    yi[j] = ok ? A(yv[j].y) : A(0);
  }
  A hr[P], hi[P];

  // z_t = y_t - sum_k L[t][t-k] z_{t-k}; h[k-1] = z_{t-k} (the z_{t-1} term last)
#define STFD_TS_FWD_ROW(j)                                   \
  A zr = yr[j], zi = yi[j];                                  \
  _Pragma("unroll") for (int k = P; k >= 1; --k) {           \
    zr = fma(-lr[j][k - 1], hr[k - 1], zr);                  \
    zr = fma(li[j][k - 1], hi[k - 1], zr);                   \
    zi = fma(-lr[j][k - 1], hi[k - 1], zi);                  \
    zi = fma(-li[j][k - 1], hr[k - 1], zi);                  \
  }                                                          \
  _Pragma("unroll") for (int k = P - 1; k >= 1; --k) {       \
    hr[k] = hr[k - 1];                                       \
    hi[k] = hi[k - 1];                                       \
  }                                                          \
  hr[0] = zr;                                                \
  hi[0] = zi;

  // x_t = w_t - sum_k conj(L[t+k][t]) x_{t+k}; h[k-1] = x_{t+k} (the x_{t+1} term last)
#define STFD_TS_BWD_ROW(j)                                                      \
  A xr = yr[j], xi = yi[j];                                                     \
  _Pragma("unroll") for (int k = P; k >= 1; --k) {                              \
    const int q = j + k;                                                        \
    const A cr = q < LEN ? lr[q < LEN ? q : 0][k - 1] : nlr[q < LEN ? 0 : q - LEN][k - 1]; \
    const A ci = q < LEN ? li[q < LEN ? q : 0][k - 1] : nli[q < LEN ? 0 : q - LEN][k - 1]; \
    xr = fma(-cr, hr[k - 1], xr);                                               \
    xr = fma(-ci, hi[k - 1], xr);                                               \
    xi = fma(-cr, hi[k - 1], xi);                                               \
    xi = fma(ci, hr[k - 1], xi);                                                \
  }                                                                             \
  _Pragma("unroll") for (int k = P - 1; k >= 1; --k) {                          \
    hr[k] = hr[k - 1];                                                          \
    hi[k] = hi[k - 1];                                                          \
  }                                                                             \
  hr[0] = xr;                                                                   \
  hi[0] = xi;

  // (1) forward sweep from a zero history -> local tail
#pragma unroll
  for (int k = 0; k < P; ++k) hr[k] = hi[k] = A(0);
#pragma unroll
  for (int j = 0; j < LEN; ++j) {
    STFD_TS_FWD_ROW(j)
  }
  // (2) reduced forward recurrence over the segments, then history = true tail of segment s-1.
  // Transfer Tf[a][c]: response of z_{t0+LEN-1-a} to the history z_{t0-1-c} = 1 (the others 0),
  // from P homogeneous sweeps over the segment's rows of L, one column at a time, parked in LDS
  // (each lane reads back only its own entries) so that one sweep state is live at a time.
  {
#pragma unroll 1
    for (int c = 0; c < P && FLY; ++c) {
      A gr[P], gi[P];
#pragma unroll
      for (int k = 0; k < P; ++k) {
        gr[k] = k == c ? A(1) : A(0);
        gi[k] = A(0);
      }
#pragma unroll
      for (int j = 0; j < LEN; ++j) {
        A zr = A(0), zi = A(0);
#pragma unroll
        for (int k = P; k >= 1; --k) {
          zr = fma(-lr[j][k - 1], gr[k - 1], zr);
          zr = fma(li[j][k - 1], gi[k - 1], zr);
          zi = fma(-lr[j][k - 1], gi[k - 1], zi);
          zi = fma(-li[j][k - 1], gr[k - 1], zi);
        }
#pragma unroll
        for (int k = P - 1; k >= 1; --k) {
          gr[k] = gr[k - 1];
          gi[k] = gi[k - 1];
        }
        gr[0] = zr;
        gi[0] = zi;
      }
#pragma unroll
      for (int a = 0; a < P; ++a) {
        A2 v;
        v.x = gr[a];
        v.y = gi[a];
        Tsh[(a * P + c) * kTsLanes + g.pl] = v;
      }
    }
#pragma unroll
    for (int a = 0; a < P; ++a)
#pragma unroll
      for (int c = 0; c < P; ++c) {
        const A2 v = FLY ? Tsh[(a * P + c) * kTsLanes + g.pl] : Tfb[(a * P + c) * kTsLanes + lane];
        tfr[a][c] = v.x;
        tfi[a][c] = v.y;
      }
    A cr0[P], ci0[P];
#pragma unroll
    for (int a = 0; a < P; ++a) {
      cr0[a] = hr[a];
      ci0[a] = hi[a];
    }
    for (int r = 1; r < segs; ++r) {
      A pr[P], pi[P];
#pragma unroll
      for (int c = 0; c < P; ++c) {
        const A vr = __shfl_up(hr[c], 1), vi = __shfl_up(hi[c], 1);
        pr[c] = s > 0 ? vr : A(0);
        pi[c] = s > 0 ? vi : A(0);
      }
#pragma unroll
      for (int a = 0; a < P; ++a) {
        A ar = cr0[a], ai = ci0[a];
#pragma unroll
        for (int c = 0; c < P; ++c) {
          ar = fma(tfr[a][c], pr[c], ar);
          ar = fma(-tfi[a][c], pi[c], ar);
          ai = fma(tfr[a][c], pi[c], ai);
          ai = fma(tfi[a][c], pr[c], ai);
        }
        hr[a] = ar;
        hi[a] = ai;
      }
    }
#pragma unroll
    for (int c = 0; c < P; ++c) {
      const A vr = __shfl_up(hr[c], 1), vi = __shfl_up(hi[c], 1);
      hr[c] = s > 0 ? vr : A(0);
      hi[c] = s > 0 ? vi : A(0);
    }
  }
  // (3) forward sweep from the true history; w = z / D in place of y
#pragma unroll
  for (int j = 0; j < LEN; ++j) {
    STFD_TS_FWD_ROW(j)
    if constexpr (!FACTOR) dv[j] = Db[j * kTsLanes + lane];
    else dv[j] = Dsh[j * kTsLanes + g.pl];
    yr[j] = zr * dv[j];
    yi[j] = zi * dv[j];
  }
  // (4) backward sweep from a zero future -> local head
#pragma unroll
  for (int k = 0; k < P; ++k) hr[k] = hi[k] = A(0);
#pragma unroll
  for (int j = LEN - 1; j >= 0; --j) {
    STFD_TS_BWD_ROW(j)
  }
  // (5) reduced backward recurrence, then future = true head of segment s+1.
  // Transfer Tb[a][c]: response of x_{t0+a} to the future x_{t0+LEN+c} = 1 (the others 0), from P
  // homogeneous backward sweeps (the rows of L past the segment come from the next lane), parked
  // in LDS like Tf.
  {
#pragma unroll 1
    for (int c = 0; c < P && FLY; ++c) {
      A gr[P], gi[P];
#pragma unroll
      for (int k = 0; k < P; ++k) {
        gr[k] = k == c ? A(1) : A(0);
        gi[k] = A(0);
      }
#pragma unroll
      for (int j = LEN - 1; j >= 0; --j) {
        A xr = A(0), xi = A(0);
#pragma unroll
        for (int k = P; k >= 1; --k) {
          const int q = j + k;
          const A cr = q < LEN ? lr[q < LEN ? q : 0][k - 1] : nlr[q < LEN ? 0 : q - LEN][k - 1];
          const A ci = q < LEN ? li[q < LEN ? q : 0][k - 1] : nli[q < LEN ? 0 : q - LEN][k - 1];
          xr = fma(-cr, gr[k - 1], xr);
          xr = fma(-ci, gi[k - 1], xr);
          xi = fma(-cr, gi[k - 1], xi);
          xi = fma(ci, gr[k - 1], xi);
        }
#pragma unroll
        for (int k = P - 1; k >= 1; --k) {
          gr[k] = gr[k - 1];
          gi[k] = gi[k - 1];
        }
        gr[0] = xr;
        gi[0] = xi;
      }
#pragma unroll
      for (int a = 0; a < P; ++a) {
        A2 v;
        v.x = gr[a];
        v.y = gi[a];
        Tsh[(a * P + c) * kTsLanes + g.pl] = v;
      }
    }
#pragma unroll
    for (int a = 0; a < P; ++a)
#pragma unroll
      for (int c = 0; c < P; ++c) {
        const A2 v = FLY ? Tsh[(a * P + c) * kTsLanes + g.pl] : Tbb[(a * P + c) * kTsLanes + lane];
        tbr[a][c] = v.x;
        tbi[a][c] = v.y;
      }
    A cr0[P], ci0[P];
#pragma unroll
    for (int a = 0; a < P; ++a) {
      cr0[a] = hr[a];
      ci0[a] = hi[a];
    }
    for (int r = 1; r < segs; ++r) {
      A pr[P], pi[P];
#pragma unroll
      for (int c = 0; c < P; ++c) {
        const A vr = __shfl_down(hr[c], 1), vi = __shfl_down(hi[c], 1);
        pr[c] = has_next ? vr : A(0);
        pi[c] = has_next ? vi : A(0);
      }
#pragma unroll
      for (int a = 0; a < P; ++a) {
        A ar = cr0[a], ai = ci0[a];
#pragma unroll
        for (int c = 0; c < P; ++c) {
          ar = fma(tbr[a][c], pr[c], ar);
          ar = fma(-tbi[a][c], pi[c], ar);
          ai = fma(tbr[a][c], pi[c], ai);
          ai = fma(tbi[a][c], pr[c], ai);
        }
        hr[a] = ar;
        hi[a] = ai;
      }
    }
#pragma unroll
    for (int c = 0; c < P; ++c) {
      const A vr = __shfl_down(hr[c], 1), vi = __shfl_down(hi[c], 1);
      hr[c] = has_next ? vr : A(0);
      hi[c] = has_next ? vi : A(0);
    }
  }
  // (6) backward sweep from the true future; write x
#pragma unroll
  for (int j = LEN - 1; j >= 0; --j) {
    STFD_TS_BWD_ROW(j)
    const int t = t0 + j;
    if (live && t < n_t) {
      T2 o;
      o.x = T(xr);
      o.y = T(xi);
      yb[t] = o;
    }
  }
#undef STFD_TS_FWD_ROW
#undef STFD_TS_BWD_ROW
}

template <typename T, typename A, int P, int LEN, int MODE>
__global__ __launch_bounds__(kTsLanes) void time_solve_kernel(T* y, const A* Lf, const A* Df, const A* Tf,
                                                            const A* Tb, const A* Sf, const A* Hb, const A* Mu,
                                                            int n_t, int segs, int mpb, int64_t N_s,
                                                            int64_t blocks_per_rhs, const int* done) {
  using A2 = typename TsVec<A>::t;
  using T2 = typename TsVec<T>::t;
  constexpr bool FACTOR = TsMode<MODE>::kFactor;
  const int64_t rhs = blockIdx.x / blocks_per_rhs;
  if (done && done[rhs]) return;
  const int64_t blk = blockIdx.x - rhs * blocks_per_rhs;
  const int lane = threadIdx.x;
  const int m = lane / segs;
  const int64_t mode = blk * mpb + m;
  const bool live = m < mpb && mode < N_s;
  __shared__ A2 Tsh[P * P * kTsLanes];            // the lanes' transfer matrices, [a][c][lane]
  __shared__ A Dsh[FACTOR ? LEN * kTsLanes : 1];  // factor form: the lanes' 1/D rows, [j][lane]
  TsLaneArgs<T, A> g;
  g.yb = reinterpret_cast<T2*>(y) + (rhs * N_s + (live ? mode : 0)) * int64_t(n_t);
  g.live = live;
  g.s = lane - m * segs;
  g.segs = segs;
  g.n_t = n_t;
  g.tl = g.pl = lane;
  g.Lf = Lf ? Lf + blk * int64_t(2 * LEN * P * kTsLanes) : nullptr;
  g.Df = Df ? Df + blk * int64_t(LEN * kTsLanes) : nullptr;
  g.Tf = Tf ? Tf + blk * int64_t(2 * P * P * kTsLanes) : nullptr;
  g.Tb = Tb ? Tb + blk * int64_t(2 * P * P * kTsLanes) : nullptr;
  g.Sf = Sf ? Sf + blk * int64_t(P * P * kTsLanes) : nullptr;
  g.Hb = Hb;
  g.mu = (FACTOR && live) ? Mu[mode] : A(0);
  g.Tsh = Tsh;
  g.Dsh = Dsh;
  time_solve_lane<T, A, P, LEN, MODE>(g);
}

// ---------------------------------------------------------------------------
// Last direction fused with the time solves (Algorithm 1: the forward product along x_d, step 3
// and the backward product along x_d in one launch).  The products along x_d and the time solves
// act on the spatial column (m_1 .. m_{d-1}) alone: the n_d rows of 2 n_t reals of one column,
// X[j][2t + c], are all that the three steps read and write.  One block per column and
// right-hand side loads them once into LDS (the slab), then
//   (1) forward product Y[m][.] = sum_j U'_f[j][m] X[j][.], MFMA tiles (16 modes x 16 reals),
//       results kept in registers until every wave has read the slab, then written over it;
//   (2) time solves of the column's n_d modes, H_i x_i = y_i in place in the slab, the lanes laid
//       out as in time_solve_kernel (mpb modes of `segs` segments per wave); the tables are stored
//       in a layout of their own (block = column * waves + wave) so that each wave reads whole
//       table lines;
//   (3) backward product Z[j][.] = sum_m U'_b[m][j] Y[m][.] from the slab, stored to global memory.
// The tensor crosses HBM once each way instead of three times, and the intermediate never leaves
// the CU.  LDS: the slab (n_d rows, ld reals each), the packed backward operand, and one region
// holding first the packed forward operand, then the waves' transfer / pivot parking of the time
// solve.  FP64 products solve in FP64; FP32 products store the slab in FP32 and solve in FP32
// with the FP32 tables (the rounding points of the three-launch path).  Every MFMA chain runs its
// K steps in the order of the mode-product kernels, so with the same segment length the result
// equals the three-launch path bit for bit.
// ---------------------------------------------------------------------------
struct FusedTimeArgs {
  const void* in;   // tensor after the forward products of x_1 .. x_{d-1}
  void* out;        // may equal in (each block reads its column before it writes it)
  const void* Uf;   // packed forward operand of x_d (fragment order, mode_product_ks K steps)
  const void* Ub;   // packed backward operand of x_d
  int n;            // n_d
  int n_t;
  int ld;           // slab row stride (reals), even and >= 2 n_t; the MFMA tiles of a row run to
                    // the next multiple of 16 (into the next row, or the operand after the last
                    // one: such columns feed only outputs that are not stored)
  int ks;           // K steps of the packed operands
  int segs, mpb;    // time-solve lane layout
  int64_t n_cols;   // columns per right-hand side (N_s / n_d)
  size_t u_bytes;   // bytes of one packed operand
  size_t park_off;  // byte offset of the parking region (after the slab and the backward operand)
  const int* done;
  const void* Lf;   // time-solve tables in the fused layout (the form's unused ones null)
  const void* Df;
  const void* Tf;
  const void* Tb;
  const void* Sf;
  const void* Hb;
  const void* Mu;   // indexed by spatial mode
};

constexpr int kFusedTiles = 8;    // output tiles (16 x 16) per wave and product at most (even)
constexpr int kFusedLoads = 12;   // complex slab entries loaded per thread at most
constexpr int kFusedULoads = 20;  // packed operand values staged per thread and operand at most

template <int PREC, typename T, int P, int LEN, int MODE, int NW>
__global__ __launch_bounds__(NW * 64) void fused_time_kernel(FusedTimeArgs a) {
  static_assert(PREC != MP_BF16, "the fused form runs the FP64 and FP32 products");
  using Tr = MPTraits<PREC>;
  using op_t = typename Tr::op_t;
  using u_t = typename Tr::u_t;
  using acc_t = typename Tr::acc_t;
  using T2 = typename TsVec<T>::t;
  constexpr int K = Tr::K;
  extern __shared__ __align__(16) unsigned char fz_smem[];
  const int64_t col = blockIdx.x, rhs = blockIdx.y;
  if (a.done && a.done[rhs]) return;  // uniform per block
  const int n = a.n, n_t = a.n_t, ld = a.ld, KS = a.ks;
  const int KS4 = (KS + 3) / 4 * 4;  // K steps staged in LDS (zeros past KS)
  const int W = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col16 = lane & 15, grp = lane >> 4;
  const int64_t row = 2 * int64_t(n_t), inner = a.n_cols * row;
  T* S = reinterpret_cast<T*>(fz_smem);
  u_t* Ubs = reinterpret_cast<u_t*>(fz_smem + size_t(n) * ld * sizeof(T));
  unsigned char* park = fz_smem + a.park_off;  // forward operand, then the time-solve parking
  u_t* Ufs = reinterpret_cast<u_t*>(park);
  const T2* src = reinterpret_cast<const T2*>(static_cast<const T*>(a.in) + rhs * int64_t(n) * inner + col * row);
  T* dst = static_cast<T*>(a.out) + rhs * int64_t(n) * inner + col * row;

  // (0) the slab and both packed operands ([group][K step, padded to KS4][lane]), every load of a
  // thread issued before its first store
  {
    const int ncplx = n * n_t;
    const int nu = int(a.u_bytes / sizeof(u_t));  // G * KS4 * 64
    const u_t* Ufg = static_cast<const u_t*>(a.Uf);
    const u_t* Ubg = static_cast<const u_t*>(a.Ub);
    T2 v[kFusedLoads];
    u_t uf[kFusedULoads], ub[kFusedULoads];
#pragma unroll
    for (int u = 0; u < kFusedLoads; ++u) {
      const int i = min(int(threadIdx.x) + u * int(blockDim.x), ncplx - 1);
      const int j = i / n_t, t = i - j * n_t;
      v[u] = src[int64_t(j) * (inner / 2) + t];
    }
#pragma unroll
    for (int u = 0; u < kFusedULoads; ++u) {
      const int i = min(int(threadIdx.x) + u * int(blockDim.x), nu - 1);
      const int gk = i >> 6, g = gk / KS4, ks = gk - g * KS4;
      const int src_i = ((g * KS + min(ks, KS - 1)) << 6) + (i & 63);
      uf[u] = ks < KS ? Ufg[src_i] : u_t(0);
      ub[u] = ks < KS ? Ubg[src_i] : u_t(0);
    }
#pragma unroll
    for (int u = 0; u < kFusedLoads; ++u) {
      const int i = int(threadIdx.x) + u * int(blockDim.x);
      if (i < ncplx) {
        const int j = i / n_t, t = i - j * n_t;
        reinterpret_cast<T2*>(S + j * ld)[t] = v[u];
      }
    }
#pragma unroll
    for (int u = 0; u < kFusedULoads; ++u) {
      const int i = int(threadIdx.x) + u * int(blockDim.x);
      if (i < nu) {
        Ufs[i] = uf[u];
        Ubs[i] = ub[u];
      }
    }
    // padding reals of every row: zeros (they feed only padding outputs, never stored)
    const int padc = ld - int(row);
    for (int i = threadIdx.x; i < n * padc; i += blockDim.x) {
      const int j = i / padc;
      S[j * ld + int(row) + (i - j * padc)] = T(0);
    }
  }
  __syncthreads();

  const int G = (n + 15) / 16, CT = int(row + 15) / 16, ntiles = G * CT;
  // two MFMA chains at once (tiles t0, t1 < ntiles): D[16 g + m][16 ct + c] = sum_k U'[k][16 g + m]
  // B[k][16 ct + c], B from the slab; four K steps of operands loaded per round, the zero steps
  // past KS add exact zeros
  auto chain2 = [&](const u_t* Us, int t0, int t1, acc_t& c0, acc_t& c1) {
    c0 = acc_t{0, 0, 0, 0};
    c1 = acc_t{0, 0, 0, 0};
    const int g0 = t0 / CT, g1 = t1 / CT;
    const u_t* U0 = Us + g0 * KS4 * 64 + lane;
    const u_t* U1 = Us + g1 * KS4 * 64 + lane;
    const T* B0 = S + 16 * (t0 - g0 * CT) + col16;
    const T* B1 = S + 16 * (t1 - g1 * CT) + col16;
    for (int k4 = 0; k4 < KS4; k4 += 4) {
      u_t ua0[4], ua1[4];
      T b0[4], b1[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = min((k4 + e) * K + grp, n - 1);
        ua0[e] = U0[(k4 + e) * 64];
        ua1[e] = U1[(k4 + e) * 64];
        b0[e] = B0[k * ld];
        b1[e] = B1[k * ld];
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const bool in_k = (k4 + e) * K + grp < n;
        const op_t x0 = to_op<PREC>(in_k ? b0[e] : T(0)), x1 = to_op<PREC>(in_k ? b1[e] : T(0));
        if constexpr (PREC == MP_F64) {
          c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ua0[e], x0, c0, 0, 0, 0);
          c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ua1[e], x1, c1, 0, 0, 0);
        } else {
          c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ua0[e], x0, c0, 0, 0, 0);
          c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ua1[e], x1, c1, 0, 0, 0);
        }
      }
    }
  };
  // (1) forward product into registers, then over the slab
  {
    acc_t acc[kFusedTiles];
#pragma unroll
    for (int q = 0; q < kFusedTiles; q += 2) {
      const int t0 = wave + q * W, t1 = wave + (q + 1) * W;
      if (t0 < ntiles) chain2(Ufs, t0, min(t1, ntiles - 1), acc[q], acc[q + 1]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kFusedTiles; ++q) {
      const int tile = wave + q * W;
      if (tile < ntiles) {
        const int g = tile / CT, ct = tile % CT;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = 16 * g + (PREC == MP_F64 ? 4 * v + grp : 4 * grp + v);
          if (m < n && 16 * ct + col16 < row) S[m * ld + 16 * ct + col16] = T(acc[q][v]);
        }
      }
    }
  }
  __syncthreads();
  // (2) time solves of the column's modes, in place in the slab
  {
    using A2 = typename TsVec<T>::t;
    const int segs = a.segs, mpb = a.mpb;
    const int ml = lane / segs;
    const int m = wave * mpb + ml;
    const bool live = ml < mpb && m < n;
    const int64_t blk = col * W + wave;
    TsLaneArgs<T, T> g;
    g.yb = reinterpret_cast<T2*>(S + (live ? m : 0) * ld);
    g.live = live;
    g.s = lane - ml * segs;
    g.segs = segs;
    g.n_t = n_t;
    g.tl = g.pl = lane;
    const T* Lf = static_cast<const T*>(a.Lf);
    const T* Df = static_cast<const T*>(a.Df);
    const T* Tf = static_cast<const T*>(a.Tf);
    const T* Tb = static_cast<const T*>(a.Tb);
    const T* Sf = static_cast<const T*>(a.Sf);
    g.Lf = Lf ? Lf + blk * int64_t(2 * LEN * P * kTsLanes) : nullptr;
    g.Df = Df ? Df + blk * int64_t(LEN * kTsLanes) : nullptr;
    g.Tf = Tf ? Tf + blk * int64_t(2 * P * P * kTsLanes) : nullptr;
    g.Tb = Tb ? Tb + blk * int64_t(2 * P * P * kTsLanes) : nullptr;
    g.Sf = Sf ? Sf + blk * int64_t(P * P * kTsLanes) : nullptr;
    g.Hb = static_cast<const T*>(a.Hb);
    g.mu = (TsMode<MODE>::kFactor && live) ? static_cast<const T*>(a.Mu)[col + a.n_cols * m] : T(0);
    // parking of this wave: transfers [P * P][64] (transfers computed), then pivots [LEN][64]
    // (factor computed)
    constexpr size_t kTsh = TsMode<MODE>::kFlyTransfers ? P * P * kTsLanes * sizeof(A2) : 0;
    constexpr size_t kDsh = TsMode<MODE>::kFactor ? LEN * kTsLanes * sizeof(T) : 0;
    unsigned char* pw = park + size_t(wave) * (kTsh + kDsh);
    g.Tsh = reinterpret_cast<A2*>(pw);
    g.Dsh = reinterpret_cast<T*>(pw + kTsh);
    time_solve_lane<T, T, P, LEN, MODE>(g);
  }
  __syncthreads();
  // (3) backward product from the slab to global memory, two tiles per round
  for (int t0 = wave; t0 < ntiles; t0 += 2 * W) {
    const int t1 = t0 + W;
    acc_t acc[2];
    chain2(Ubs, t0, min(t1, ntiles - 1), acc[0], acc[1]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int tile = h ? t1 : t0;
      const int g = tile / CT, c = 16 * (tile - g * CT) + col16;
      if (tile < ntiles && c < row) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = 16 * g + (PREC == MP_F64 ? 4 * v + grp : 4 * grp + v);
          if (j < n) dst[int64_t(j) * inner + c] = T(acc[h][v]);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Time solves on time axes longer than the segmented layouts hold (more than 64 segments of the
// longest compiled length): one lane per mode runs the banded forward and backward substitutions
// over the whole axis, L D L^H x = y with the host factors in their mode-fastest layout
// Lfac[t][k-1][mode] (complex) and 1/D[t][mode] (loads coalesced across the lanes).  Dependent
// chain 2 n_t steps; used for the long time axes of the one-dimensional problems only.
// ---------------------------------------------------------------------------
// [rhs][mode][t] <-> [rhs][t][mode] through 32 x 32 LDS tiles (both sides coalesced).
template <typename T2>
__global__ __launch_bounds__(256) void time_transpose_kernel(const T2* in, T2* out, int64_t rows, int64_t cols) {
  __shared__ T2 tile[32][33];
  const int64_t rhs = blockIdx.z;
  const T2* src = in + rhs * rows * cols;
  T2* dst = out + rhs * rows * cols;
  const int64_t r0 = int64_t(blockIdx.y) * 32, c0 = int64_t(blockIdx.x) * 32;
  for (int k = threadIdx.y; k < 32; k += 8) {
    const int64_t r = r0 + k, c = c0 + threadIdx.x;
    if (r < rows && c < cols) tile[k][threadIdx.x] = src[r * cols + c];
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += 8) {
    const int64_t c = c0 + k, r = r0 + threadIdx.x;
    if (r < rows && c < cols) dst[c * rows + r] = tile[threadIdx.x][k];
  }
}

template <typename T, int P>
__global__ __launch_bounds__(256) void time_solve_seq_kernel(T* y, const T* Lfac, const T* Dinv, int n_t,
                                                             int64_t N_s, const int* done) {
  using T2 = typename TsVec<T>::t;
  const int64_t rhs = blockIdx.y;
  if (done && done[rhs]) return;
  const int64_t mode = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (mode >= N_s) return;
  // y of one right-hand side transposed to [t][mode] (time_transpose_kernel): the lanes' rows are
  // adjacent in memory
  struct Rows {
    T2* p;
    int64_t s;
    __device__ T2& operator[](int t) const { return p[int64_t(t) * s]; }
  } yb{reinterpret_cast<T2*>(y) + rhs * N_s * int64_t(n_t) + mode, N_s};
  const T2* L = reinterpret_cast<const T2*>(Lfac);
  T hr[P], hi[P];
#pragma unroll
  for (int k = 0; k < P; ++k) hr[k] = hi[k] = T(0);
  // z_t = y_t - sum_k L[t][t-k] z_{t-k}; w_t = z_t / D_t in place (h[k-1] = z_{t-k})
  for (int t = 0; t < n_t; ++t) {
    const T2 yv = yb[t];
    T zr = yv.x, zi = yv.y;
#pragma unroll
    for (int k = P; k >= 1; --k) {
      const T2 l = t - k >= 0 ? L[(int64_t(t) * P + (k - 1)) * N_s + mode] : T2{T(0), T(0)};
      zr = fma(-l.x, hr[k - 1], zr);
      zr = fma(l.y, hi[k - 1], zr);
      zi = fma(-l.x, hi[k - 1], zi);
      zi = fma(-l.y, hr[k - 1], zi);
    }
#pragma unroll
    for (int k = P - 1; k >= 1; --k) {
      hr[k] = hr[k - 1];
      hi[k] = hi[k - 1];
    }
    hr[0] = zr;
    hi[0] = zi;
    const T d = Dinv[int64_t(t) * N_s + mode];
    T2 w;
    w.x = zr * d;
    w.y = zi * d;
    yb[t] = w;
  }
  // x_t = w_t - sum_k conj(L[t+k][t]) x_{t+k} (h[k-1] = x_{t+k})
#pragma unroll
  for (int k = 0; k < P; ++k) hr[k] = hi[k] = T(0);
  for (int t = n_t - 1; t >= 0; --t) {
    const T2 wv = yb[t];
    T xr = wv.x, xi = wv.y;
#pragma unroll
    for (int k = P; k >= 1; --k) {
      const T2 l = t + k < n_t ? L[(int64_t(t + k) * P + (k - 1)) * N_s + mode] : T2{T(0), T(0)};
      xr = fma(-l.x, hr[k - 1], xr);
      xr = fma(-l.y, hi[k - 1], xr);
      xi = fma(-l.x, hi[k - 1], xi);
      xi = fma(l.y, hr[k - 1], xi);
    }
#pragma unroll
    for (int k = P - 1; k >= 1; --k) {
      hr[k] = hr[k - 1];
      hi[k] = hi[k - 1];
    }
    hr[0] = xr;
    hi[0] = xi;
    T2 xo;
    xo.x = xr;
    xo.y = xi;
    yb[t] = xo;
  }
}

// ---------------------------------------------------------------------------
// Matvec of one-dimensional problems with long time axes (the stencil kernel stages a whole
// time line per point in LDS, which bounds n_t): one lane per (x_1 point, t) entry sums the
// (2 p_s + 1)(2 p_t + 1) neighbours of eq. syst_mat directly,
//   Y(t, i) = sum_s sum_dt (S_1[i][s] L_t + S_2[i][s] M_t + i S_3[i][s] K_t)[t][dt] X(t + dt - p_t, i + s - p_s),
// neighbours through L1 / L2 (consecutive lanes read consecutive t), and one partial of
// Re <x, y> per block.
// ---------------------------------------------------------------------------
constexpr int kMvLongBlock = 256;
__global__ __launch_bounds__(kMvLongBlock) void matvec_long1d_kernel(const double* x, double* y, const double* Sc,
                                                                    const double* TbL, int n_t, int pt, int n1,
                                                                    int ps, int64_t blocks_per_rhs,
                                                                    double* partial, const int* done) {
  __shared__ double red[kMvLongBlock / 64];
  const int64_t rhs = blockIdx.y;
  if (done && done[rhs]) return;
  const int64_t N = int64_t(n1) * n_t;
  const int64_t e = int64_t(blockIdx.x) * kMvLongBlock + threadIdx.x;
  const bool active = e < N;
  const int64_t ec = active ? e : N - 1;
  const int i = int(ec / n_t), t = int(ec - int64_t(i) * n_t);
  const int ws = 2 * ps + 1, wt = 2 * pt + 1;
  const double2* X = reinterpret_cast<const double2*>(x) + rhs * N;
  double yr = 0.0, yi = 0.0;
  for (int s = 0; s < ws; ++s) {
    const int j = i + s - ps;
    if (j < 0 || j >= n1) continue;
    const double c1 = Sc[(int64_t(i) * ws + s) * 3], c2 = Sc[(int64_t(i) * ws + s) * 3 + 1],
                 c3 = Sc[(int64_t(i) * ws + s) * 3 + 2];
    for (int dt = 0; dt < wt; ++dt) {
      const int tt = t + dt - pt;
      if (tt < 0 || tt >= n_t) continue;
      const double* tb = TbL + (int64_t(t) * wt + dt) * 4;
      const double ar = fma(c1, tb[0], c2 * tb[1]), ai = c3 * tb[2];  // S_1 L_t + S_2 M_t + i S_3 K_t
      const double2 xv = X[int64_t(j) * n_t + tt];
      yr = fma(ar, xv.x, fma(-ai, xv.y, yr));
      yi = fma(ar, xv.y, fma(ai, xv.x, yi));
    }
  }
  double part = 0.0;
  if (active) {
    reinterpret_cast<double2*>(y)[rhs * N + e] = make_double2(yr, yi);
    const double2 xe = X[e];
    part = xe.x * yr + xe.y * yi;
  }
  if (partial) {
    part = wave_sum(part);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t2 = 0.0;
      for (int w = 0; w < kMvLongBlock / 64; ++w) t2 += red[w];
      partial[rhs * blocks_per_rhs + blockIdx.x] = t2;
    }
  }
}

// ---------------------------------------------------------------------------
// Matrix-free system matvec (Section 5.3, eq. syst_mat with potential terms):
//   Y = sum_k T_k X S_k^T, X viewed as n_t x N_s (time fastest).
// Lanes run over the flat (spatial point, t) index of X, so that no lane idles
// whatever n_t is; a block covers K whole spatial points (K n_t lanes) so that
// the time coupling of phase 2 stays inside the block.
// Phase 1: Z_k(t, i) = sum_s S_k[i][s] X(t, i + o(s)).  The block's
//          coefficients S_k[i][s] are staged in LDS (the lanes of one point
//          read one address: broadcast); each neighbour value is one 16-byte
//          bounds-checked buffer load at a per-lane byte offset summed from
//          per-axis offsets computed once; a neighbour outside the grid gets an
//          offset beyond the buffer, which the load returns as zero.
// Phase 2: Y(t, i) = sum_k sum_dt T_k[t][dt] Z_k(t + dt, i) with T_3 = i K_t,
//          Z from LDS (in the space of the coefficients, after a barrier) and
//          the bands from LDS, zero outside 0 <= t + dt < n_t.
// Optionally writes one partial of Re <x, y> per block (PCG's <p, A p>).
// ---------------------------------------------------------------------------
constexpr int kMvMaxNt = 128;      // longest time axis of the stencil and sum-factorised matvecs
// one-dimensional problems beyond those limits (long axes): the chunked mode product, the
// sequential time solve and the direct matvec
constexpr int kLongMaxN = 1024;    // n_1 at most
constexpr int kLongMaxNt = 2048;   // n_t at most
constexpr int kMvLanes = 512;      // lanes per matvec block at most
constexpr size_t kMvLds = 48 * 1024;  // LDS per block for coefficients / Z (several blocks per CU)
constexpr uint32_t kMvBadOffset = 1u << 30;  // neighbour outside the grid (beyond any buffer)

struct MatvecArgs {
  const double* x;
  double* y;
  const double* Sc;     // [N_s][stencil][3] interleaved spatial coefficients
  const double* TbL;    // time bands in the kernel's LDS layout [n_t][2 pt + 1][4]: L_t, M_t, K_t, 0
  int n_t, pt;
  int n1, n2, n3;
  int K;                // spatial points per block
  int64_t N_s;
  int64_t blocks_per_rhs;
  int64_t nrhs;
  int64_t xcd_span;     // logical blocks per XCD
  double* partial;      // [rhs][blocks_per_rhs] or nullptr
  const int* done;
};

typedef unsigned int mv_u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 mv_load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  const mv_u4 v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
  double2 o;
  o.x = __builtin_bit_cast(double, (unsigned long long)v.x | ((unsigned long long)v.y << 32));
  o.y = __builtin_bit_cast(double, (unsigned long long)v.z | ((unsigned long long)v.w << 32));
  return o;
}

template <int D, int PS, int PT, int RB>
__global__ __launch_bounds__(kMvLanes) void matvec_kernel(MatvecArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[kMvLanes / 64];
  constexpr int W = 2 * PS + 1;
  constexpr int ST = (D == 1 ? W : (D == 2 ? W * W : W * W * W));
  constexpr int WT = 2 * PT + 1;
  const int tid = threadIdx.x;
  // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
  // contiguous range of spatial points so that its L2 holds one slab of X.
  const int64_t lb = int64_t(blockIdx.x % kXcds) * a.xcd_span + blockIdx.x / kXcds;
  if (lb >= a.blocks_per_rhs * a.nrhs) return;
  const int64_t rhs = lb / a.blocks_per_rhs;
  const int64_t blk = lb - rhs * a.blocks_per_rhs;
  if (a.done && a.done[rhs]) return;
  STFD_STAMP(0, 0);
  const int n_t = a.n_t, K = a.K;
  const int64_t i0 = blk * K;
  const int kp = int(min<int64_t>(K, a.N_s - i0));
  double* Cs = reinterpret_cast<double*>(smem_raw);  // [K][ST][3]; later Z: [K][n_t][3] complex
  const size_t area = (max(size_t(K) * ST * 3, size_t(K) * n_t * 6) + 1) / 2 * 2;
  double2* Tb = reinterpret_cast<double2*>(Cs + area);  // [n_t][WT][2] double2: (L_t, M_t), (K_t, 0)
  // staging: all loads of a thread are issued before its LDS stores (one memory round trip)
  {
    constexpr int kBatch = 4;
    const int nc = kp * ST * 3, nb = n_t * WT * 2;
    const double* src = a.Sc + i0 * (ST * 3);
    const double2* tsrc = reinterpret_cast<const double2*>(a.TbL);
    for (int b0 = 0; b0 < max(nc, nb); b0 += int(blockDim.x) * kBatch) {
      double cv[kBatch];
      double2 tv[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int idx = b0 + u * int(blockDim.x) + tid;
        cv[u] = src[min(idx, nc - 1)];
        tv[u] = tsrc[min(idx, nb - 1)];
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int idx = b0 + u * int(blockDim.x) + tid;
        if (idx < nc) Cs[idx] = cv[u];
        if (idx < nb) Tb[idx] = tv[u];
      }
    }
  }
  __syncthreads();
  STFD_STAMP(0, 1);
  const int pl = tid / n_t;             // point of this lane within the block
  const int t = tid - pl * n_t;
  const bool active = pl < kp;
  const int pc = min(pl, kp - 1);
  const int64_t i = i0 + pc;
  const double* X = a.x + rhs * a.N_s * int64_t(2 * n_t);
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(X), 0, int(a.N_s * n_t * 16), 0x00020000);
  // byte offsets of the neighbours along x_1 (kMvBadOffset outside the grid), per lane
  const int i1 = int(i % a.n1);
  const int64_t q = i / a.n1;
  const int i2 = (D >= 2) ? int(q % a.n2) : 0;
  const int i3 = (D >= 3) ? int(q / a.n2) : 0;
  uint32_t off1[W];
#pragma unroll
  for (int o = 0; o < W; ++o) {
    const int j1 = i1 + o - PS;
    off1[o] = (j1 >= 0 && j1 < a.n1) ? uint32_t((j1 * n_t + t) * 16) : kMvBadOffset;
  }
  const uint32_t s2 = uint32_t(a.n1 * n_t * 16), s3 = uint32_t(a.n2) * s2;
  // byte offset of stencil row r = (o_3, o_2) (x_2 offset fastest)
  auto row_off = [&](int r) -> uint32_t {
    if constexpr (D == 1) {
      return 0u;
    } else if constexpr (D == 2) {
      const int j2 = i2 + r - PS;
      return (j2 >= 0 && j2 < a.n2) ? uint32_t(j2) * s2 : kMvBadOffset;
    } else {
      const int j2 = i2 + r % W - PS, j3 = i3 + r / W - PS;
      return (j2 >= 0 && j2 < a.n2 && j3 >= 0 && j3 < a.n3) ? uint32_t(j2) * s2 + uint32_t(j3) * s3 : kMvBadOffset;
    }
  };
  double z[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const double* C = Cs + size_t(pc) * ST * 3;
  constexpr int NROWS = ST / W;
  // N stencil rows from r0: all N*W loads are issued together, then used
  auto rows = [&](auto nrows, int r0) {
    constexpr int N = decltype(nrows)::value;
    double2 v[N][W];
#pragma unroll
    for (int rr = 0; rr < N; ++rr) {
      const uint32_t ro = row_off(r0 + rr);
#pragma unroll
      for (int o = 0; o < W; ++o) v[rr][o] = mv_load(rs, ro + off1[o]);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int rr = 0; rr < N; ++rr)
#pragma unroll
      for (int o = 0; o < W; ++o) {
        const int sidx = (r0 + rr) * W + o;
        const double c0 = C[sidx * 3], c1 = C[sidx * 3 + 1], c2 = C[sidx * 3 + 2];
        z[0] = fma(c0, v[rr][o].x, z[0]); z[1] = fma(c0, v[rr][o].y, z[1]);
        z[2] = fma(c1, v[rr][o].x, z[2]); z[3] = fma(c1, v[rr][o].y, z[3]);
        z[4] = fma(c2, v[rr][o].x, z[4]); z[5] = fma(c2, v[rr][o].y, z[5]);
      }
  };
  constexpr int NB = NROWS / RB, REM = NROWS % RB;
#pragma unroll 1
  for (int b = 0; b < NB; ++b) rows(std::integral_constant<int, RB>(), b * RB);
  if constexpr (REM > 0) rows(std::integral_constant<int, (REM > 0 ? REM : 1)>(), NB * RB);
  STFD_STAMP(0, 2);
  __syncthreads();  // every lane is done with the coefficients: Z takes their space
  double2* Zs = reinterpret_cast<double2*>(Cs);
  if (active) {
#pragma unroll
    for (int k = 0; k < 3; ++k) Zs[tid * 3 + k] = make_double2(z[2 * k], z[2 * k + 1]);
  }
  __syncthreads();
  double part = 0.0;
  if (active) {
    double yr = 0.0, yi = 0.0;
    const int base = pl * n_t;
#pragma unroll
    for (int dt = 0; dt < WT; ++dt) {
      const int tt = min(max(t + dt - PT, 0), n_t - 1);
      const double2 tlm = Tb[(t * WT + dt) * 2], tk = Tb[(t * WT + dt) * 2 + 1];
      const double2 z0 = Zs[(base + tt) * 3], z1 = Zs[(base + tt) * 3 + 1], z2 = Zs[(base + tt) * 3 + 2];
      yr += tlm.x * z0.x + tlm.y * z1.x - tk.x * z2.y;
      yi += tlm.x * z0.y + tlm.y * z1.y + tk.x * z2.x;
    }
    const int64_t g = (rhs * a.N_s + i) * n_t + t;
    reinterpret_cast<double2*>(a.y)[g] = make_double2(yr, yi);
    if (a.partial) {
      const double2 xc = reinterpret_cast<const double2*>(a.x)[g];
      part = xc.x * yr + xc.y * yi;  // Re(conj(x) y)
    }
  }
  STFD_STAMP(0, 3);
  if (a.partial) {
    part = wave_sum(part);
    const int w = tid >> 6, nw = int(blockDim.x) >> 6;
    if ((tid & 63) == 0) red[w] = part;
    __syncthreads();
    if (tid == 0) {
      double sum = 0.0;
      for (int k = 0; k < nw; ++k) sum += red[k];
      a.partial[rhs * a.blocks_per_rhs + blk] = sum;
    }
  }
}

// ---------------------------------------------------------------------------
// BLAS-1 kernels of PCG.  Vectors are complex FP64 [rhs][N]; grid = (kVecGrid, nrhs).
// Scalar state per right-hand side lives in PcgScalars.
// ---------------------------------------------------------------------------
struct PcgScalars {
  double nf2;       // ||f||^2
  double rz[2];     // <r_k, z_k> by iteration parity
  double res;       // ||r_k|| / ||f||
  double true_res;
  int iters;
  int status;
  int done;
  int kcur;  // iteration index of the iteration in flight (set by pcg_update_xr)
  double x0_scale;  // factor applied to a given initial guess (0: cold start)
};

// partial sums of Re<a, b> (and optionally Re<a, c>) over this block's range
__global__ __launch_bounds__(kVecBlock) void dot2_kernel(const double* a, const double* b, const double* c,
                                                          int64_t n2, double* pb, double* pc, const int* done) {
  __shared__ double sh[kVecBlock / 64];
  const int rhs = blockIdx.y;
  if (done && done[rhs]) return;
  const double* A = a + rhs * n2;
  const double* B = b + rhs * n2;
  const double* C = c ? c + rhs * n2 : nullptr;
  double sb = 0.0, sc = 0.0;
  for (int64_t k = (int64_t(blockIdx.x) * kVecBlock + threadIdx.x) * 2; k < n2; k += int64_t(gridDim.x) * kVecBlock * 2) {
    const double ar = A[k], ai = A[k + 1];
    sb += ar * B[k] + ai * B[k + 1];
    if (C) sc += ar * C[k] + ai * C[k + 1];
  }
  sb = block_sum<kVecBlock>(sb, sh);
  if (threadIdx.x == 0) pb[rhs * gridDim.x + blockIdx.x] = sb;
  if (C) {
    sc = block_sum<kVecBlock>(sc, sh);
    if (threadIdx.x == 0) pc[rhs * gridDim.x + blockIdx.x] = sc;
  }
}

// r = f - q (given x0) or r = f (zero x0, also zeroes x); partial ||f||^2
__global__ __launch_bounds__(kVecBlock) void pcg_init_kernel(const double* f, const double* q, double* r,
                                                              double* x, int64_t n2, double* pf) {
  __shared__ double sh[kVecBlock / 64];
  const int rhs = blockIdx.y;
  const double* F = f + rhs * n2;
  double* R = r + rhs * n2;
  double s = 0.0;
  for (int64_t k = (int64_t(blockIdx.x) * kVecBlock + threadIdx.x) * 2; k < n2; k += int64_t(gridDim.x) * kVecBlock * 2) {
    const double fr = F[k], fi = F[k + 1];
    s += fr * fr + fi * fi;
    if (q) {
      R[k] = fr - q[rhs * n2 + k];
      R[k + 1] = fi - q[rhs * n2 + k + 1];
    } else {
      R[k] = fr;
      R[k + 1] = fi;
      x[rhs * n2 + k] = 0.0;
      x[rhs * n2 + k + 1] = 0.0;
    }
  }
  s = block_sum<kVecBlock>(s, sh);
  if (threadIdx.x == 0) pf[rhs * gridDim.x + blockIdx.x] = s;
}

// partial sums of <x, f> (real and imaginary part) and Re<x, q> over this block's range
__global__ __launch_bounds__(kVecBlock) void dot_x0_kernel(const double* x, const double* f, const double* q,
                                                            int64_t n2, double* pre, double* pim, double* pq) {
  __shared__ double sh[kVecBlock / 64];
  const int rhs = blockIdx.y;
  const double* X = x + rhs * n2;
  const double* F = f + rhs * n2;
  const double* Q = q + rhs * n2;
  double sr = 0.0, si = 0.0, sq = 0.0;
  for (int64_t k = (int64_t(blockIdx.x) * kVecBlock + threadIdx.x) * 2; k < n2; k += int64_t(gridDim.x) * kVecBlock * 2) {
    const double xr = X[k], xi = X[k + 1];
    sr += xr * F[k] + xi * F[k + 1];  // conj(x) f
    si += xr * F[k + 1] - xi * F[k];
    sq += xr * Q[k] + xi * Q[k + 1];
  }
  sr = block_sum<kVecBlock>(sr, sh);
  if (threadIdx.x == 0) pre[rhs * gridDim.x + blockIdx.x] = sr;
  si = block_sum<kVecBlock>(si, sh);
  if (threadIdx.x == 0) pim[rhs * gridDim.x + blockIdx.x] = si;
  sq = block_sum<kVecBlock>(sq, sh);
  if (threadIdx.x == 0) pq[rhs * gridDim.x + blockIdx.x] = sq;
}

// scalar bookkeeping after the initial residual: ||f||^2, ||r_0||, convergence at k = 0
// Energy-optimal scaling of a given initial guess: with q = A x0, the complex factor
// alpha = <x0, f> / <x0, q> minimises ||u - alpha x0||_A over complex multiples (u = A^{-1} f; it
// corrects the modulus and the phase of a guess); <x0, q> <= 0 or a non-finite value gives
// alpha = 0, the cold start.  x <- alpha x, r = f - alpha q, partials of ||f||^2; the scalar
// state records |alpha|.
__global__ __launch_bounds__(kVecBlock) void pcg_x0_scale_kernel(const double* f, const double* q, double* r,
                                                                  double* x, int64_t n2, const double* pxf_re,
                                                                  const double* pxf_im, const double* pxq, int nparts,
                                                                  double* pf, PcgScalars* sc) {
  __shared__ double sh[kVecBlock / 64];
  const int rhs = blockIdx.y;
  const double xfr = sum_partials<kVecBlock>(pxf_re + rhs * nparts, nparts, sh);
  const double xfi = sum_partials<kVecBlock>(pxf_im + rhs * nparts, nparts, sh);
  const double xq = sum_partials<kVecBlock>(pxq + rhs * nparts, nparts, sh);
  double ar = xfr / xq, ai = xfi / xq;
  if (!(xq > 0.0) || !std::isfinite(ar) || !std::isfinite(ai)) ar = ai = 0.0;
  const double* F = f + rhs * n2;
  const double* Q = q + rhs * n2;
  double* R = r + rhs * n2;
  double* X = x + rhs * n2;
  double s = 0.0;
  for (int64_t k = (int64_t(blockIdx.x) * kVecBlock + threadIdx.x) * 2; k < n2; k += int64_t(gridDim.x) * kVecBlock * 2) {
    const double fr = F[k], fi = F[k + 1];
    s += fr * fr + fi * fi;
    const double qr = Q[k], qi = Q[k + 1], xr = X[k], xi = X[k + 1];
    R[k] = fr - (ar * qr - ai * qi);
    R[k + 1] = fi - (ar * qi + ai * qr);
    X[k] = ar * xr - ai * xi;
    X[k + 1] = ar * xi + ai * xr;
  }
  s = block_sum<kVecBlock>(s, sh);
  if (threadIdx.x == 0) pf[rhs * gridDim.x + blockIdx.x] = s;
  if (blockIdx.x == 0 && threadIdx.x == 0) sc[rhs].x0_scale = std::sqrt(ar * ar + ai * ai);
}
// A scaled initial guess whose residual exceeds ||f|| is dropped: x = 0, r = f (the cold start),
// so the residual-based stopping test never starts behind the cold start either.
__global__ __launch_bounds__(kVecBlock) void pcg_x0_revert_kernel(const double* f, double* r, double* x, int64_t n2,
                                                                   const PcgScalars* sc) {
  const int rhs = blockIdx.y;
  const PcgScalars st = sc[rhs];
  if (st.x0_scale == 0.0 || !(st.res > 1.0)) return;
  for (int64_t k = int64_t(blockIdx.x) * kVecBlock + threadIdx.x; k < n2; k += int64_t(gridDim.x) * kVecBlock) {
    r[rhs * n2 + k] = f[rhs * n2 + k];
    x[rhs * n2 + k] = 0.0;
  }
}
// second half of the revert (a separate launch: the kernel above reads the flags it clears here)
__global__ void pcg_x0_revert_finish_kernel(PcgScalars* sc, int* done, int nrhs, double tol) {
  const int rhs = blockIdx.x * blockDim.x + threadIdx.x;
  if (rhs >= nrhs) return;
  PcgScalars& st = sc[rhs];
  if (st.x0_scale == 0.0 || !(st.res > 1.0)) return;
  st.x0_scale = 0.0;
  st.res = 1.0;
  st.done = (1.0 <= tol) ? 1 : 0;
  done[rhs] = st.done;
}
__global__ __launch_bounds__(kVecBlock) void pcg_start_kernel(const double* pf, const double* prr, int nparts,
                                                               PcgScalars* sc, int* done, double tol, int* ctr,
                                                               int x0_mode) {
  __shared__ double sh[kVecBlock / 64];
  const int rhs = blockIdx.x;
  if (rhs == 0 && threadIdx.x == 0) ctr[0] = 0;
  const double nf2 = sum_partials<kVecBlock>(pf + rhs * nparts, nparts, sh);
  const double rr = prr ? sum_partials<kVecBlock>(prr + rhs * nparts, nparts, sh) : nf2;
  if (threadIdx.x == 0) {
    PcgScalars& s = sc[rhs];
    s.nf2 = nf2;
    s.iters = 0;
    s.kcur = 0;
    if (x0_mode != 2) s.x0_scale = (x0_mode == 1) ? 1.0 : 0.0;
    s.status = STFD_OK;
    s.done = 0;
    s.rz[0] = s.rz[1] = 0.0;
    s.true_res = 0.0;
    if (!(nf2 > 0.0) || !std::isfinite(nf2)) {
      // f = 0: the solution is u = 0 (already in x for a zero start)
      s.res = 0.0;
      s.done = 1;
      if (!std::isfinite(nf2)) s.status = STFD_EBREAKDOWN;
    } else {
      s.res = sqrt(rr / nf2);
      if (!std::isfinite(s.res)) { s.status = STFD_EBREAKDOWN; s.done = 1; }
      else if (s.res <= tol) s.done = 1;
    }
    done[rhs] = s.done;
  }
}

// p = z; rz[0] = <r, z>
__global__ __launch_bounds__(kVecBlock) void pcg_first_p_kernel(const double* z, double* p, int64_t n2,
                                                                 const double* prz, int nparts, PcgScalars* sc,
                                                                 int* done) {
  __shared__ double sh[kVecBlock / 64];
  const int rhs = blockIdx.y;
  if (done[rhs]) return;
  const double rz = sum_partials<kVecBlock>(prz + rhs * nparts, nparts, sh);
  for (int64_t k = (int64_t(blockIdx.x) * kVecBlock + threadIdx.x) * 2; k < n2; k += int64_t(gridDim.x) * kVecBlock * 2) {
    p[rhs * n2 + k] = z[rhs * n2 + k];
    p[rhs * n2 + k + 1] = z[rhs * n2 + k + 1];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[rhs].rz[0] = rz;
    if (!(rz > 0.0) || !std::isfinite(rz)) {
      sc[rhs].status = STFD_EBREAKDOWN;
      sc[rhs].done = 1;
      done[rhs] = 1;
    }
  }
}

// alpha = rz / <p, q>; x += alpha p; r -= alpha q; partial ||r||^2.  Every load the update
// depends on (done flag, rz, this thread's share of the <p, q> partials and its first (p, q, r, x)
// quadruple) is issued in one batch ahead of the block sum: one memory round trip before the
// update instead of a chain of four.  Blocks of a finished right-hand side load and then leave.
__global__ __launch_bounds__(kVecBlock) void pcg_update_xr_kernel(const double* p, const double* q, double* x,
                                                                   double* r, int64_t n2, const double* ppq,
                                                                   int npq, PcgScalars* sc, int parity,
                                                                   double* prr, const int* done, int* ctr) {
  __shared__ double sh[kVecBlock / 64];
  const int rhs = blockIdx.y, tid = threadIdx.x;
  // launch counter of this solve (read by pcg_end_iter to pick its host ring slot)
  if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) ctr[0] += 1;
  const double2* pc = reinterpret_cast<const double2*>(p + rhs * n2);
  const double2* qc = reinterpret_cast<const double2*>(q + rhs * n2);
  double2* xc = reinterpret_cast<double2*>(x + rhs * n2);
  double2* rc = reinterpret_cast<double2*>(r + rhs * n2);
  const int64_t m = n2 / 2, stride = int64_t(gridDim.x) * kVecBlock;
  const int64_t k0 = int64_t(blockIdx.x) * kVecBlock + tid;
  const double* pp = ppq + int64_t(rhs) * npq;
  // partials: lanes past the count load nothing (exec mask); the vector address is clamped
  const int dn = done[rhs];
  const double rz = sc[rhs].rz[parity];
  const int iters = sc[rhs].iters;
  double v[kSumBatch];
#pragma unroll
  for (int u = 0; u < kSumBatch; ++u) {
    const int idx = u * kVecBlock + tid;
    v[u] = idx < npq ? pp[idx] : 0.0;
  }
  const int64_t kc = min(k0, m - 1);
  double2 rv = rc[kc], qv = qc[kc], pv = pc[kc], xv = xc[kc];
  load_batch_end();
  double t = v[0];
#pragma unroll
  for (int u = 1; u < kSumBatch; ++u) t += v[u];
  for (int idx = kSumBatch * kVecBlock + tid; idx < npq; idx += kVecBlock) t += pp[idx];
  const double pq = block_sum<kVecBlock>(t, sh);
  if (dn) return;
  const bool ok = (pq > 0.0) && std::isfinite(pq);
  const double alpha = ok ? rz / pq : 0.0;
  if (blockIdx.x == 0 && tid == 0) sc[rhs].kcur = iters;
  double s = 0.0;
  for (int64_t k = k0; k < m; k += stride) {
    if (k != k0) {
      rv = rc[k];
      qv = qc[k];
      pv = pc[k];
      xv = xc[k];
    }
    const double rr = rv.x - alpha * qv.x, ri = rv.y - alpha * qv.y;
    if (ok) {
      rc[k] = make_double2(rr, ri);
      xc[k] = make_double2(xv.x + alpha * pv.x, xv.y + alpha * pv.y);
    }
    s += rr * rr + ri * ri;
  }
  s = block_sum<kVecBlock>(s, sh);
  if (tid == 0) prr[rhs * gridDim.x + blockIdx.x] = ok ? s : NAN;
}

// End of iteration k for one right-hand side: convergence / breakdown / iteration-limit test on
// ||r_{k+1}|| (partials of pcg_update_xr), then beta = (<r, z_new> - <r, z_old>) / rz_k (partials
// of the last mode product) and p = z_new + beta p.  Every block sums every partial in the same
// order (kEndBlock threads, one batch of loads that also holds the state and this thread's first
// (z, p) pair) and so takes the same decision; block 0 records the state, the per-rhs done flag
// and a copy in host-mapped memory.  Block 0 writes only what the other blocks do not read, and
// the done flag it may raise only skips the direction update, which a finished system does not
// need.  With kEndBlock threads per block the sums are those of a single-block reduction.
constexpr int kEndBlock = 1024;
constexpr int kEndGrid = 256;
__global__ __launch_bounds__(kEndBlock) void pcg_end_iter_kernel(const double* znew, double* p, int64_t n2,
                                                                  const double* prr, int nrr, const double* pa,
                                                                  const double* pb, int nab, PcgScalars* sc,
                                                                  int parity, int* done, int maxit, double tol,
                                                                  PcgScalars* host_ring, int ring_stride,
                                                                  const int* ctr) {
  constexpr int NT = kEndBlock, NW = NT / 64;
  __shared__ double sh[3 * NW];
  const int rhs = blockIdx.y, tid = threadIdx.x;
  const double* a = prr + int64_t(rhs) * nrr;
  const double* b = pa + int64_t(rhs) * nab;
  const double* c = pb + int64_t(rhs) * nab;
  const double2* zc = reinterpret_cast<const double2*>(znew + rhs * n2);
  double2* pc = reinterpret_cast<double2*>(p + rhs * n2);
  const int64_t m = n2 / 2, stride = int64_t(gridDim.x) * NT;
  const int64_t k0 = int64_t(blockIdx.x) * NT + tid;
  // ||r||^2, <r, z_new>, <r, z_old>: the first batch of partials (lanes past a count load
  // nothing), the done flag, the ring counter, the state and this thread's first (z, p) pair in
  // one batch of loads; further batches only for more than NT * kSumBatch partials
  double va[kSumBatch], vb[kSumBatch], vc[kSumBatch];
#pragma unroll
  for (int u = 0; u < kSumBatch; ++u) {
    const int idx = u * NT + tid;
    va[u] = idx < nrr ? a[idx] : 0.0;
    vb[u] = idx < nab ? b[idx] : 0.0;
    vc[u] = idx < nab ? c[idx] : 0.0;
  }
  const int dn = done[rhs];
  const int cnt = ctr[0];
  const double nf2 = sc[rhs].nf2;
  const double rzk = parity ? sc[rhs].rz[1] : sc[rhs].rz[0];
  const int k = sc[rhs].kcur;
  const int64_t kc = min(k0, m - 1);
  double2 zv = zc[kc], pv = pc[kc];
  load_batch_end();
  PcgScalars* host_slot = host_ring ? host_ring + ((cnt - 1) % kLag) * ring_stride : nullptr;
  if (dn) {
    if (blockIdx.x == 0 && tid == 0 && host_slot) host_slot[rhs] = sc[rhs];
    return;
  }
  double ta = va[0], tb = vb[0], tc = vc[0];
#pragma unroll
  for (int u = 1; u < kSumBatch; ++u) {
    ta += va[u];
    tb += vb[u];
    tc += vc[u];
  }
  for (int idx = NT * kSumBatch + tid; idx < max(nrr, nab); idx += NT) {
    ta += idx < nrr ? a[idx] : 0.0;
    tb += idx < nab ? b[idx] : 0.0;
    tc += idx < nab ? c[idx] : 0.0;
  }
  ta = wave_sum(ta);
  tb = wave_sum(tb);
  tc = wave_sum(tc);
  if ((tid & 63) == 0) {
    sh[tid >> 6] = ta;
    sh[NW + (tid >> 6)] = tb;
    sh[2 * NW + (tid >> 6)] = tc;
  }
  __syncthreads();
  double rr = 0.0, rzn_all = 0.0, rzm = 0.0;
  for (int i = 0; i < NW; ++i) {
    rr += sh[i];
    rzn_all += sh[NW + i];
    rzm += sh[2 * NW + i];
  }
  const double res = sqrt(rr / nf2);
  int status = STFD_OK;
  bool finished = false;
  double rzn = 0.0, beta = 0.0;
  if (!std::isfinite(res)) {
    status = STFD_EBREAKDOWN;
    finished = true;
  } else if (res <= tol) {
    finished = true;
  } else if (k + 1 >= maxit) {
    status = STFD_NOT_CONVERGED;
    finished = true;
  } else {
    rzn = rzn_all;
    if (!(rzn > 0.0) || !std::isfinite(rzn) || !std::isfinite(rzm)) {
      status = STFD_EBREAKDOWN;
      finished = true;
    } else {
      beta = (rzn - rzm) / rzk;
    }
  }
  if (!finished) {
    for (int64_t q = k0; q < m; q += stride) {
      if (q != k0) {
        zv = zc[q];
        pv = pc[q];
      }
      pc[q] = make_double2(zv.x + beta * pv.x, zv.y + beta * pv.y);
    }
  }
  if (blockIdx.x == 0 && tid == 0) {
    PcgScalars& st = sc[rhs];
    st.iters = k + 1;
    if (std::isfinite(res)) st.res = res;
    // (constant indices only: a dynamic index would keep the state in scratch memory)
    if (parity) st.rz[0] = rzn;
    else st.rz[1] = rzn;
    st.status = status;
    st.done = finished ? 1 : 0;
    done[rhs] = st.done;
    if (host_slot) host_slot[rhs] = st;
  }
}

// ||f - q||^2 partials (true residual with q = A x)
__global__ __launch_bounds__(kVecBlock) void resid_norm_kernel(const double* f, const double* q, int64_t n2, double* pr) {
  __shared__ double sh[kVecBlock / 64];
  const int rhs = blockIdx.y;
  double s = 0.0;
  for (int64_t k = (int64_t(blockIdx.x) * kVecBlock + threadIdx.x) * 2; k < n2; k += int64_t(gridDim.x) * kVecBlock * 2) {
    const int64_t g = rhs * n2 + k;
    const double a = f[g] - q[g], b = f[g + 1] - q[g + 1];
    s += a * a + b * b;
  }
  s = block_sum<kVecBlock>(s, sh);
  if (threadIdx.x == 0) pr[rhs * gridDim.x + blockIdx.x] = s;
}

__global__ __launch_bounds__(kVecBlock) void pcg_finish_kernel(const double* pr, int nparts, PcgScalars* sc) {
  __shared__ double sh[kVecBlock / 64];
  const int rhs = blockIdx.x;
  const double rr = sum_partials<kVecBlock>(pr + rhs * nparts, nparts, sh);
  if (threadIdx.x == 0) sc[rhs].true_res = (sc[rhs].nf2 > 0.0) ? sqrt(rr / sc[rhs].nf2) : 0.0;
}

// diagnostic: one MFMA of each kind with A[m][k] = m + 16 k, B[k][n] = (k == n % K)
__global__ void mfma_layout_kernel(double* o64, float* o32, float* obf) {
  const int l = threadIdx.x;
  const int m = l & 15, g = l >> 4;
  d4_t a64 = {0, 0, 0, 0};
  a64 = __builtin_amdgcn_mfma_f64_16x16x4f64(double(m + 16 * g), double(g == (m & 3)), a64, 0, 0, 0);
  f4_t a32 = {0, 0, 0, 0};
  a32 = __builtin_amdgcn_mfma_f32_16x16x4f32(float(m + 16 * g), float(g == (m & 3)), a32, 0, 0, 0);
  s4_t av, bv;
  for (int e = 0; e < 4; ++e) {
    const int k = 4 * g + e;
    av[e] = f32_to_bf16(float(m + 16 * k));
    bv[e] = f32_to_bf16(float(k == (m & 15)));
  }
  f4_t abf = {0, 0, 0, 0};
  abf = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, abf, 0, 0, 0);
  for (int v = 0; v < 4; ++v) {
    o64[l * 4 + v] = a64[v];
    o32[l * 4 + v] = a32[v];
    obf[l * 4 + v] = abf[v];
  }
}

}  // namespace stfd

// ===========================================================================
// Host side: the problem handle and the C ABI
// ===========================================================================
struct stfd_problem {
  stfd::HostProblem hp;
  int max_nrhs = 1;
  int64_t n2 = 0;  // reals per vector (2 N)
  // device data
  // mode-product operands packed in fragment order, per precision (MP_F64 / MP_F32 / MP_BF16) and
  // direction: forward U'[j][a] = U[j][a] (apply U^T), backward U'[j][a] = U[a][j] (apply U)
  void* Upk_fwd[3][3] = {};
  void* Upk_bwd[3][3] = {};
  int64_t upk_slice[3] = {0, 0, 0};  // packed elements per x_1 slice (mapped domain), per precision
  // segmented time-solve tables (layout: TimeSolvePlan in host_setup.h)
  double* TsL = nullptr;
  double* TsS = nullptr;   // factor-in-kernel form: segment entry states, time bands, nu lambda_i
  double* TsH = nullptr;
  double* TsMu = nullptr;
  float* TsS32 = nullptr;
  float* TsH32 = nullptr;
  float* TsMu32 = nullptr;
  double* TsTf = nullptr;  // segment transfers (small grids only, else null)
  double* TsTb = nullptr;
  double* TsD = nullptr;
  float* TsL32 = nullptr;
  float* TsTf32 = nullptr;
  float* TsTb32 = nullptr;  // FP32 copies for the FP32 / BF16 applies
  float* TsD32 = nullptr;
  int ts_len = 0, ts_segs = 0, ts_mpb = 0;
  int64_t ts_blocks = 0;
  // last direction fused with the time solves (fused_time_kernel): tables in the fused layout
  // (the form's used ones; Mu indexed by spatial mode), launch shape, and whether applies use it
  double* FzL = nullptr;
  double* FzD = nullptr;
  double* FzTf = nullptr;
  double* FzTb = nullptr;
  double* FzS = nullptr;
  double* FzH = nullptr;
  double* FzMu = nullptr;
  float* FzL32 = nullptr;
  float* FzD32 = nullptr;
  float* FzTf32 = nullptr;
  float* FzTb32 = nullptr;
  float* FzS32 = nullptr;
  float* FzH32 = nullptr;
  float* FzMu32 = nullptr;
  int fz_len = 0, fz_mode = 0, fz_nw = 0, fz_waves = 0, fz_segs = 0, fz_mpb = 0;
  bool fz_on = false;
  double* Sc = nullptr;
  double* TbL = nullptr;  // time bands in the matvec's LDS layout
  double* work64[2] = {nullptr, nullptr};
  float* work32[2] = {nullptr, nullptr};
  double* vec[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // r, z, z2, p, q
  double* parts = nullptr;  // 6 partial arrays of max_nrhs * max_parts
  int64_t max_parts = 0;
  stfd::PcgScalars* sc = nullptr;
  int* done = nullptr;
  int* ctr = nullptr;  // iterations launched in the current solve (device)
  stfd::PcgScalars* sc_host = nullptr;  // pinned host ring [kLag][max_nrhs], written by kernels
  // stream and events of this handle's job in a batched solve (created on first use)
  hipStream_t job_stream = nullptr;
  hipEvent_t job_ev[stfd::kLag + 1] = {};
  stfd::PcgScalars* sc_host_dev = nullptr;  // device address of sc_host
  int64_t mp_last_blocks[3] = {0, 0, 0};  // per precision: blocks per rhs of the last mode product (dot partials)
  int mp_rt[3][3] = {};                   // [precision][direction]: row groups per wave of the mode products
  int ts_mode = 0;                        // time solve: 0 tables, 1 transfers computed, 2 factor computed,
                                          // 3 one lane per mode over the whole axis (TsL / TsD hold the
                                          // host factors in their mode-fastest layout)
  bool autotuned = false;
  double tune_ms = 0.0;                   // device time spent by the setup's tuning runs
  int64_t u_slice0 = 0;                  // per-mode pencils along x_1 (mapped domain): n_1^2, else 0
  int64_t mv_blocks = 0;
  int mv_points = 1;  // spatial points per matvec block
  bool mv_long = false;  // one-dimensional problem with a long time axis: matvec_long1d_kernel
  size_t max_lds = 65536;  // per-block LDS limit of the device used at setup
  int n_cus = 256;         // compute units of the device used at setup
  stfd::LoadPlan load;     // basis matrices on the Gauss grids (right-hand side assembly)
  stfd::Geometry geom;
  stfd::SpatialModel model;   // weighted terms of the spatial factors (potential, geometry)
  stfd::SpatialDevice sdev;   // device basis tables, base stencils and model arrays
  int* lift_status_host = nullptr;  // pinned: status of the last lifting CG, written by the device
  int* lift_status_dev = nullptr;   // device address of lift_status_host
  int lift_max_iter = 200;          // iteration limit of the lifting CG
  double* rhs_work = nullptr;       // load-vector scratch for one right-hand side (setup), or nullptr
  double* rhs_lift = nullptr;       // lifting tensors of max_nrhs right-hand sides (setup), or nullptr
  bool sf_on = false;               // the matvec runs sum-factorised (no stencils are stored)
  stfd::SumFacPlan sf;
  std::vector<void*> allocs;
  // captured PCG iterations (STFD_PCG_GRAPH), kept for later solves with the same arguments: the
  // two graph executables of one job (iteration parities) and what their kernels were captured with
  struct CachedIterations {
    const double* f = nullptr;
    double* x = nullptr;
    int64_t nrhs = 0;
    int precision = 0, maxit = 0;
    double rtol = 0.0;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    uint64_t used = 0;
  };
  std::vector<CachedIterations> graphs;
  uint64_t graph_clock = 0;
  // HIP-event timing of the mode-product launches (stfd_timing_begin / stfd_timing_end)
  bool timing = false;
  std::vector<hipEvent_t> tev;  // start/end pairs, recorded on the launch stream
  size_t tev_used = 0;
};

namespace stfd {

static void graph_cache_clear(stfd_problem* P);  // drops the captured PCG iterations of a handle

template <typename T>
static int dev_alloc(stfd_problem* P, T** ptr, size_t count) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) {
    g_last_hip_error = int(e);
    return STFD_ENOMEM;
  }
  P->allocs.push_back(p);
  *ptr = static_cast<T*>(p);
  return STFD_OK;
}

template <typename T>
static int upload(stfd_problem* P, T** ptr, const T* src, size_t count) {
  int rc = dev_alloc(P, ptr, count);
  if (rc) return rc;
  STFD_HIP(hipMemcpy(*ptr, src, count * sizeof(T), hipMemcpyHostToDevice));
  return STFD_OK;
}

// 16-row groups per mode-product wave.  Two (one U' load serves both MFMA chains, In rows are
// read 32 values at a time) when the launch is large enough to keep the chip busy with half the
// waves and n <= 80 (two FP64 chains of more K steps would spill); else one.  Measured: 3D p = 3
// 48^4 (67k one-group waves per product) apply FP64 619 -> 603 us, FP32 457 -> 428 us, BF16 417
// -> 375 us; 2D 64^3 (2960 waves) 38.7 -> 41.8 us, hence the threshold.  Depends on per-rhs
// sizes only, so every precision writes the same dot partials.
constexpr int64_t kMpTwoGroupMinWaves = 16384;
// Output columns computed by vector FMAs instead of an MFMA group of their own (the kernels'
// remainder columns): the last r of n = 16 g + r, g >= 1, r <= 2, in FP64 and FP32 launches large
// enough to keep the chip busy with the fewer waves (as for two row groups); none for the long
// directions.  In a small launch the longer waves of the last group set the time (2D 64^3: 6.8 ->
// 7.3 us per product), in a large one the saved MFMA work does (3D 48^4 FP64 apply 461 -> 420 us,
// FP32 308 -> 288 us).  BF16 keeps the MFMA group: its MFMA is cheap and rounding the operands to
// BF16 on the vector units is not (3D 48^4 apply 262 -> 283 us).  Depends on the precision and
// per-rhs sizes only, so every shape and every batch size computes the same way.
static int mode_product_rem(int prec, int n, int64_t inner, int64_t outer_per_rhs) {
  const int r = n - 16 * ((n + 15) / 16 - 1);
  const int64_t waves1 = int64_t((n + 15) / 16) * outer_per_rhs * ((inner + 15) / 16);
  return (prec != MP_BF16 && n > 16 && n <= kMaxModeN && r <= 2 && waves1 >= kMpTwoGroupMinWaves) ? r : 0;
}
// 16-column groups computed by MFMA chains
static int mode_product_groups(int prec, int n, int64_t inner, int64_t outer_per_rhs) {
  return (n + 15) / 16 - (mode_product_rem(prec, n, inner, outer_per_rhs) > 0 ? 1 : 0);
}
static int mode_product_row_groups(int n, int64_t inner, int64_t outer_per_rhs) {
  const int64_t waves1 = int64_t((n + 15) / 16) * outer_per_rhs * ((inner + 15) / 16);
  return (n <= 80 && waves1 >= kMpTwoGroupMinWaves) ? 2 : 1;
}

// Blocks (one wave each) of one right-hand side of a mode product: 16-column groups x (tiles of
// 16 RT rows of every outer slice, padded to a multiple of the XCD count).  Depends only on
// per-rhs sizes, so the number of dot partials per right-hand side is fixed.
// Launch shapes of a mode product: 1 or 2 = one column group per wave with that many 16-row groups,
// kMpWide = every column group per wave (mode_product_wide_kernel, n <= 80, one operand).
constexpr int kMpWide = 3;
constexpr int64_t kMpWideBlocks = 1024;  // blocks per right-hand side of the wide form at most
static int64_t mode_product_wide_blocks(int64_t inner, int64_t outer_per_rhs) {
  const int64_t tiles = outer_per_rhs * ((inner + 15) / 16);
  return std::min<int64_t>((tiles + 3) / 4, kMpWideBlocks);
}
static int64_t mode_product_blocks_per_rhs(int prec, int n, int64_t inner, int64_t outer_per_rhs, int rt = 0) {
  if (rt == kMpWide) return mode_product_wide_blocks(inner, outer_per_rhs);
  const int rows = 16 * (rt > 0 ? rt : mode_product_row_groups(n, inner, outer_per_rhs));
  const int64_t tiles = outer_per_rhs * ((inner + rows - 1) / rows);
  // one-group form: kMpWaves row tiles per block; long directions: one per block
  const int64_t units = n > kMaxModeN ? tiles : (tiles + kMpWaves - 1) / kMpWaves;
  return int64_t(mode_product_groups(prec, n, inner, outer_per_rhs)) * ((units + kXcds - 1) / kXcds * kXcds);
}

// K steps of one mode-product instantiation: exact for FP64 (K = 4) and BF16 (K = 16), buckets
// of 4 steps for FP32 (K = 4); the operand is packed for exactly this count
static int mode_product_ks(int prec, int n) {
  if (prec == MP_BF16) return (n + 15) / 16;
  const int nks = (n + 3) / 4;
  return prec == MP_F32 ? (nks + 3) / 4 * 4 : nks;
}

// U' (nsl slices of n x n, U'[j][a] = Uop[(k n + j) n + a]) in the order the mode-product
// lanes read it: [slice][column group][K step][lane][e] with j = ks K + E (lane / 16) + e and
// a = 16 cg + lane % 16, zero where j or a >= n.  A lane's values for one K step are E
// consecutive elements and a wave's loads cover whole, aligned cache lines (the rows of an
// n x n operand are not multiples of 128 bytes); the zeros replace the masks of the padded
// K steps and columns.
template <typename T>
static void pack_mode_operand(const double* Uop, int n, int nsl, int K, int E, int KS, std::vector<T>& out) {
  const int groups = (n + 15) / 16;
  const size_t per_slice = size_t(groups) * KS * 64 * E;
  out.assign(per_slice * nsl, T(0));
  for (int k = 0; k < nsl; ++k)
    for (int cg = 0; cg < groups; ++cg)
      for (int ks = 0; ks < KS; ++ks)
        for (int lane = 0; lane < 64; ++lane)
          for (int e = 0; e < E; ++e) {
            const int j = ks * K + E * (lane >> 4) + e, a = cg * 16 + (lane & 15);
            if (j < n && a < n)
              out[size_t(k) * per_slice + ((size_t(cg) * KS + ks) * 64 + lane) * E + e] =
                  T(Uop[(size_t(k) * n + j) * n + a]);
          }
}

// K-step counts of the instantiations whose n can have remainder columns: n = 16 g + 1 or 2 gives
// KS = 4 g + 1 (FP64), 4 (g + 1) (FP32); none in BF16
template <int PREC, int KS>
constexpr bool mode_product_has_rem() {
  return PREC == MP_F64 ? (KS % 4 == 1 && KS >= 5) : PREC == MP_F32 ? (KS % 4 == 0 && KS >= 8) : false;
}
// launch with RT row groups and RC remainder columns per wave (false: no such instantiation), U'
// staged in LDS unless the operand differs per outer slice
template <int PREC, typename Tin, typename Tout, int KS, int RT, bool DOT, int RC>
static void launch_mode_product_lds(dim3 grid, dim3 block, hipStream_t s, const ModeProductArgs& a) {
  if (a.u_slice_stride == 0)
    hipLaunchKernelGGL((mode_product_kernel<PREC, Tin, Tout, KS, RT, DOT, RC, true>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((mode_product_kernel<PREC, Tin, Tout, KS, RT, DOT, RC, false>), grid, block, 0, s, a);
}
template <int PREC, typename Tin, typename Tout, int KS, int RT, bool DOT>
static bool launch_mode_product_rc(int rc, dim3 grid, dim3 block, hipStream_t s, const ModeProductArgs& a) {
  if constexpr (mode_product_has_rem<PREC, KS>()) {
    if (rc == 1) {
      launch_mode_product_lds<PREC, Tin, Tout, KS, RT, DOT, 1>(grid, block, s, a);
      return true;
    }
    if (rc == 2) {
      launch_mode_product_lds<PREC, Tin, Tout, KS, RT, DOT, 2>(grid, block, s, a);
      return true;
    }
  }
  if (rc != 0) return false;
  launch_mode_product_lds<PREC, Tin, Tout, KS, RT, DOT, 0>(grid, block, s, a);
  return true;
}
// the two-row-group variant exists only for the K-step counts of n <= 80
// (mode_product_row_groups never asks for it beyond)
template <int PREC, typename Tin, typename Tout, int KS, bool DOT>
static bool launch_mode_product_rt_dot(int rt, int rc, dim3 grid, dim3 block, hipStream_t s,
                                       const ModeProductArgs& a) {
  constexpr bool kTwo = (PREC == MP_BF16) ? (KS <= 5) : (KS <= 20);
  if constexpr (kTwo) {
    if (rt == 2) return launch_mode_product_rc<PREC, Tin, Tout, KS, 2, DOT>(rc, grid, block, s, a);
  }
  return launch_mode_product_rc<PREC, Tin, Tout, KS, 1, DOT>(rc, grid, block, s, a);
}
// the fused dot products exist only for the FP64 output of the last backward product
template <int PREC, typename Tin, typename Tout, int KS>
static bool launch_mode_product_rt(int rt, int rc, dim3 grid, dim3 block, hipStream_t s, const ModeProductArgs& a) {
  if constexpr (std::is_same<Tout, double>::value) {
    if (a.part_a) return launch_mode_product_rt_dot<PREC, Tin, Tout, KS, true>(rt, rc, grid, block, s, a);
  }
  return launch_mode_product_rt_dot<PREC, Tin, Tout, KS, false>(rt, rc, grid, block, s, a);
}

struct DotEpilogue {
  const double* r = nullptr;
  const double* zold = nullptr;
  double* part_a = nullptr;
  double* part_b = nullptr;
};

template <int PREC, typename Tin, typename Tout>
static int launch_mode_product_wide(const void* in, void* out, const void* U, int n, int64_t inner, int64_t outer,
                                    int64_t outer_per_rhs, const int* done, hipStream_t s, const DotEpilogue& ep) {
  ModeProductArgs a;
  a.in = in;
  a.out = out;
  a.U = U;
  a.u_slice_stride = 0;
  a.n = n;
  a.inner = inner;
  a.outer = outer;
  a.outer_per_rhs = outer_per_rhs;
  a.n_row_tiles = (inner + 15) / 16;
  a.tiles_per_rhs = outer_per_rhs * a.n_row_tiles;
  a.tiles_pad = a.tiles_per_rhs;
  a.groups = mode_product_groups(PREC, n, inner, outer_per_rhs);
  a.done = done;
  a.dot_r = ep.r;
  a.dot_z = ep.zold;
  a.part_a = ep.part_a;
  a.part_b = ep.part_b;
  if (ep.part_a && !std::is_same<Tout, double>::value) return STFD_EINVAL;
  const int64_t nrhs = outer / outer_per_rhs;
  const int64_t bpr = mode_product_wide_blocks(inner, outer_per_rhs);
  if (nrhs < 1 || nrhs > 65535 || bpr < 1) return nrhs < 1 ? STFD_OK : STFD_EINVAL;
  const dim3 grid(static_cast<unsigned>(bpr), static_cast<unsigned>(nrhs)), block(256);
  const int ks = mode_product_ks(PREC, n);
  const bool dot = ep.part_a != nullptr;
  const int rc = mode_product_rem(PREC, n, inner, outer_per_rhs);
#define STFD_MPW_RC(KV, RCV)                                                                                     \
  if constexpr (std::is_same<Tout, double>::value) {                                                            \
    if (dot) {                                                                                                  \
      hipLaunchKernelGGL((mode_product_wide_kernel<PREC, Tin, Tout, KV, true, RCV>), grid, block, 0, s, a, bpr); \
      break;                                                                                                    \
    }                                                                                                           \
  }                                                                                                             \
  hipLaunchKernelGGL((mode_product_wide_kernel<PREC, Tin, Tout, KV, false, RCV>), grid, block, 0, s, a, bpr);    \
  break;
#define STFD_MPW(KV)                                          \
  case KV:                                                    \
    if constexpr (mode_product_has_rem<PREC, KV>()) {         \
      if (rc == 1) {                                          \
        STFD_MPW_RC(KV, 1)                                    \
      }                                                       \
      if (rc == 2) {                                          \
        STFD_MPW_RC(KV, 2)                                    \
      }                                                       \
    }                                                         \
    if (rc != 0) return STFD_EINVAL;                          \
    STFD_MPW_RC(KV, 0)
  if constexpr (PREC == MP_F64) {
    switch (ks) {
      STFD_MPW(1) STFD_MPW(2) STFD_MPW(3) STFD_MPW(4) STFD_MPW(5) STFD_MPW(6) STFD_MPW(7) STFD_MPW(8)
      STFD_MPW(9) STFD_MPW(10) STFD_MPW(11) STFD_MPW(12) STFD_MPW(13) STFD_MPW(14) STFD_MPW(15) STFD_MPW(16)
      STFD_MPW(17) STFD_MPW(18) STFD_MPW(19) STFD_MPW(20)
      default:
        return STFD_EINVAL;
    }
  } else if constexpr (PREC == MP_F32) {
    switch (ks) {
      STFD_MPW(4) STFD_MPW(8) STFD_MPW(12) STFD_MPW(16) STFD_MPW(20)
      default:
        return STFD_EINVAL;
    }
  } else {
    switch (ks) {
      STFD_MPW(1) STFD_MPW(2) STFD_MPW(3) STFD_MPW(4) STFD_MPW(5)
      default:
        return STFD_EINVAL;
    }
  }
#undef STFD_MPW
#undef STFD_MPW_RC
  STFD_HIP(hipGetLastError());
  return STFD_OK;
}

template <int PREC, typename Tin, typename Tout>
static int launch_mode_product(const void* in, void* out, const void* U, int n, int64_t inner, int64_t outer,
                               int64_t outer_per_rhs, const int* done, hipStream_t s,
                               const DotEpilogue& ep = DotEpilogue(), int64_t u_slice_stride = 0, int rt = 0) {
  if (n < 1 || n > kLongMaxN || outer_per_rhs < 1 || rt < 0 || rt > kMpWide || (rt >= 2 && n > 80) ||
      (rt == kMpWide && u_slice_stride != 0) || (n > kMaxModeN && (rt > 1 || u_slice_stride != 0)))
    return STFD_EINVAL;
  if (rt == kMpWide) return launch_mode_product_wide<PREC, Tin, Tout>(in, out, U, n, inner, outer, outer_per_rhs, done, s, ep);
  ModeProductArgs a;
  a.in = in;
  a.out = out;
  a.U = U;
  a.u_slice_stride = u_slice_stride;
  a.n = n;
  a.inner = inner;
  a.outer = outer;
  a.outer_per_rhs = outer_per_rhs;
  const int RTn = rt > 0 ? rt : mode_product_row_groups(n, inner, outer_per_rhs);
  a.n_row_tiles = (inner + 16 * RTn - 1) / (16 * RTn);
  a.tiles_per_rhs = outer_per_rhs * a.n_row_tiles;
  // blocks per (right-hand side, column group), padded to a multiple of the XCD count: groups of
  // kMpWaves row tiles (one-group form), single tiles (long directions)
  const bool long_dir = n > kMaxModeN;
  const int64_t units = long_dir ? a.tiles_per_rhs : (a.tiles_per_rhs + kMpWaves - 1) / kMpWaves;
  a.tiles_pad = (units + kXcds - 1) / kXcds * kXcds;
  a.groups = mode_product_groups(PREC, n, inner, outer_per_rhs);
  const int rc = mode_product_rem(PREC, n, inner, outer_per_rhs);
  a.done = done;
  a.dot_r = ep.r;
  a.dot_z = ep.zold;
  a.part_a = ep.part_a;
  if (ep.part_a && !std::is_same<Tout, double>::value) return STFD_EINVAL;  // epilogue: FP64 output only
  a.part_b = ep.part_b;
  constexpr int K = MPTraits<PREC>::K;
  const int nks = (n + K - 1) / K;
  const int64_t blocks = (outer / outer_per_rhs) * a.groups * a.tiles_pad;
  if (blocks <= 0) return STFD_OK;
  if (blocks % kXcds != 0 || blocks > int64_t(UINT32_MAX)) return STFD_EINVAL;  // the kernel's XCD remap needs it
  const dim3 grid(static_cast<unsigned>(blocks)), block(long_dir ? 64 : 64 * kMpWaves);
  if (n > kMaxModeN) {
    // long direction: K steps in chunks (the operand is packed with mode_product_ks steps)
    const int ks = mode_product_ks(PREC, n);
    if constexpr (std::is_same<Tout, double>::value) {
      if (a.part_a) {
        hipLaunchKernelGGL((mode_product_long_kernel<PREC, Tin, Tout, true>), grid, block, 0, s, a, ks);
        STFD_HIP(hipGetLastError());
        return STFD_OK;
      }
    }
    hipLaunchKernelGGL((mode_product_long_kernel<PREC, Tin, Tout, false>), grid, block, 0, s, a, ks);
    STFD_HIP(hipGetLastError());
    return STFD_OK;
  }
  // FP64: one instantiation per K-step count; FP32 (K = 4): buckets of 4 steps; BF16 (K = 16): exact
#define STFD_MP(B)                                                                                         \
  case B:                                                                                                  \
    if (!launch_mode_product_rt<PREC, Tin, Tout, (PREC == MP_F32 ? 4 * B : B)>(RTn, rc, grid, block, s, a)) \
      return STFD_EINVAL;                                                                                  \
    break;
  const int sel = PREC == MP_F32 ? (nks + 3) / 4 : nks;
  if ((PREC == MP_F32 ? 4 * sel : sel) != mode_product_ks(PREC, n)) return STFD_EINVAL;  // packing must match
  if constexpr (PREC == MP_F64) {
    switch (sel) {
      STFD_MP(1) STFD_MP(2) STFD_MP(3) STFD_MP(4) STFD_MP(5) STFD_MP(6) STFD_MP(7) STFD_MP(8)
      STFD_MP(9) STFD_MP(10) STFD_MP(11) STFD_MP(12) STFD_MP(13) STFD_MP(14) STFD_MP(15) STFD_MP(16)
      STFD_MP(17) STFD_MP(18) STFD_MP(19) STFD_MP(20) STFD_MP(21) STFD_MP(22) STFD_MP(23) STFD_MP(24)
      STFD_MP(25) STFD_MP(26) STFD_MP(27) STFD_MP(28) STFD_MP(29) STFD_MP(30) STFD_MP(31) STFD_MP(32)
      default:
        return STFD_EINVAL;
    }
  } else {
    switch (sel) {
      STFD_MP(1) STFD_MP(2) STFD_MP(3) STFD_MP(4) STFD_MP(5) STFD_MP(6) STFD_MP(7) STFD_MP(8)
      default:
        return STFD_EINVAL;
    }
  }
#undef STFD_MP
  STFD_HIP(hipGetLastError());
  return STFD_OK;
}

// reals below and slices above direction l of one right-hand side (the mode product's inner and
// outer extents)
static int64_t mp_inner(const HostProblem& hp, int l) {
  int64_t v = 2 * int64_t(hp.n_t);
  for (int k = 0; k < l; ++k) v *= hp.n_s[k];
  return v;
}
static int64_t mp_outer(const HostProblem& hp, int l) {
  int64_t v = 1;
  for (int k = l + 1; k < hp.d; ++k) v *= hp.n_s[k];
  return v;
}
// direction of the last backward product (x_1 on the unit cube, x_d on a mapped domain)
static int mp_last_dir(const stfd_problem* P) { return P->u_slice0 ? P->hp.d - 1 : 0; }
static void set_last_blocks(stfd_problem* P) {
  const int l = mp_last_dir(P);
  for (int prec = MP_F64; prec <= MP_BF16; ++prec)
    P->mp_last_blocks[prec] = mode_product_blocks_per_rhs(prec, P->hp.n_s[l], mp_inner(P->hp, l), mp_outer(P->hp, l),
                                                          P->mp_rt[prec][l]);
}
static int64_t mp_last_blocks_bound(const stfd_problem* P) {
  const int l = mp_last_dir(P);
  // BF16 has no remainder columns: the most column groups, hence blocks, of any precision
  return mode_product_blocks_per_rhs(MP_BF16, P->hp.n_s[l], mp_inner(P->hp, l), mp_outer(P->hp, l), 1);
}

// FP64 storage: FP64 solve; FP32 storage: FP32 solve with the FP32 tables
template <typename T>
static int launch_time_solve(stfd_problem* P, T* y, int64_t nrhs, const int* done, hipStream_t s, T* tmp) {
  const HostProblem& hp = P->hp;
  const int64_t bpr = P->ts_blocks;
  const dim3 grid(unsigned(bpr * nrhs)), block(kTsLanes);
  const T *L, *D, *Tf, *Tb, *S, *H, *Mu;
  if constexpr (std::is_same<T, double>::value) {
    L = P->TsL, D = P->TsD, Tf = P->TsTf, Tb = P->TsTb, S = P->TsS, H = P->TsH, Mu = P->TsMu;
  } else {
    L = P->TsL32, D = P->TsD32, Tf = P->TsTf32, Tb = P->TsTb32, S = P->TsS32, H = P->TsH32, Mu = P->TsMu32;
  }
  const int mode = P->ts_mode;
  if (mode == 3) {
    // y transposed into tmp (the apply's other intermediate), solved there, transposed back
    using T2 = typename TsVec<T>::t;
    if (nrhs < 1) return STFD_OK;
    if (!tmp || nrhs > 65535) return STFD_EINVAL;
    const dim3 tb(32, 8);
    const dim3 tg_fwd(unsigned((hp.n_t + 31) / 32), unsigned((hp.N_s + 31) / 32), unsigned(nrhs));
    const dim3 tg_bwd(unsigned((hp.N_s + 31) / 32), unsigned((hp.n_t + 31) / 32), unsigned(nrhs));
    hipLaunchKernelGGL(time_transpose_kernel<T2>, tg_fwd, tb, 0, s, reinterpret_cast<const T2*>(y),
                       reinterpret_cast<T2*>(tmp), hp.N_s, int64_t(hp.n_t));
    const dim3 sgrid(unsigned((hp.N_s + 255) / 256), unsigned(nrhs));
    switch (hp.p_t) {
#define STFD_TSQ(PV)                                                                                          \
  case PV:                                                                                                    \
    hipLaunchKernelGGL((time_solve_seq_kernel<T, PV>), sgrid, dim3(256), 0, s, tmp, L, D, hp.n_t, hp.N_s, done); \
    break;
      STFD_TSQ(1) STFD_TSQ(2) STFD_TSQ(3) STFD_TSQ(4) STFD_TSQ(5) STFD_TSQ(6)
#undef STFD_TSQ
      default:
        return STFD_EINVAL;
    }
    hipLaunchKernelGGL(time_transpose_kernel<T2>, tg_bwd, tb, 0, s, reinterpret_cast<const T2*>(tmp),
                       reinterpret_cast<T2*>(y), int64_t(hp.n_t), hp.N_s);
    STFD_HIP(hipGetLastError());
    return STFD_OK;
  }
#define STFD_TS(PV, LV)                                                                                        \
  if (hp.p_t == PV && P->ts_len == LV) {                                                                       \
    if (mode == 0)                                                                                             \
      hipLaunchKernelGGL((time_solve_kernel<T, T, PV, LV, 0>), grid, block, 0, s, y, L, D, Tf, Tb, S, H, Mu,    \
                         hp.n_t, P->ts_segs, P->ts_mpb, hp.N_s, bpr, done);                                    \
    else if (mode == 1)                                                                                        \
      hipLaunchKernelGGL((time_solve_kernel<T, T, PV, LV, 1>), grid, block, 0, s, y, L, D, Tf, Tb, S, H, Mu,    \
                         hp.n_t, P->ts_segs, P->ts_mpb, hp.N_s, bpr, done);                                    \
    else                                                                                                       \
      hipLaunchKernelGGL((time_solve_kernel<T, T, PV, LV, 2>), grid, block, 0, s, y, L, D, Tf, Tb, S, H, Mu,    \
                         hp.n_t, P->ts_segs, P->ts_mpb, hp.N_s, bpr, done);                                    \
    STFD_HIP(hipGetLastError());                                                                               \
    return STFD_OK;                                                                                            \
  }
  STFD_TS_INSTANCES
#undef STFD_TS
  return STFD_EINVAL;
}

// Fused last-direction launches (fused_time_kernel): the compiled (P, LEN, form, waves per block
// at most).  Four-wave blocks leave each wave the whole register file of its SIMD (long segments);
// eight-wave blocks take the columns whose modes need more waves.
#define STFD_FZ_INSTANCES                                                                              \
  STFD_FZ(3, 8, 2, 8) STFD_FZ(3, 16, 2, 4) STFD_FZ(4, 8, 2, 4) STFD_FZ(4, 12, 2, 4)

struct FusedShape {
  int len = 0, mode = 0, nw = 0, waves = 0, segs = 0, mpb = 0, ld = 0;
  size_t lds = 0, u_bytes = 0, park_off = 0;
};

// Launch shape of the fused form (segment length len, time-solve form mode, block bound nw) in
// precision prec; false where it does not apply or fit (waves, tiles, loads, LDS).
static bool fused_shape(const stfd_problem* P, int prec, int len, int mode, int nw, FusedShape& f) {
  const HostProblem& hp = P->hp;
  if (hp.d < 2 || P->u_slice0 || prec == MP_BF16 || len < hp.p_t) return false;
  const int n = hp.n_s[hp.d - 1], nt = hp.n_t, pt = hp.p_t;
  const int segs = (nt + len - 1) / len;
  if (segs > 64) return false;
  const int mpb = 64 / segs, waves = (n + mpb - 1) / mpb;
  if (waves > nw) return false;
  const int G = (n + 15) / 16, CT = (2 * nt + 15) / 16;
  const int ks4 = (mode_product_ks(prec, n) + 3) / 4 * 4;
  if (G * CT > kFusedTiles * waves || int64_t(n) * nt > int64_t(kFusedLoads) * waves * 64 ||
      G * ks4 * 64 > kFusedULoads * waves * 64)
    return false;
  const size_t tb = prec == MP_F64 ? sizeof(double) : sizeof(float);
  f.len = len;
  f.mode = mode;
  f.nw = nw;
  f.waves = waves;
  f.segs = segs;
  f.mpb = mpb;
  f.ld = 2 * nt;
  f.u_bytes = size_t(G) * ks4 * 64 * tb;  // one value per lane and K step, K steps padded to 4
  f.park_off = (size_t(n) * f.ld * tb + f.u_bytes + 15) / 16 * 16;
  const size_t tsh = mode >= 1 ? size_t(pt) * pt * 64 * 2 * tb : 0;
  const size_t dsh = mode == 2 ? size_t(len) * 64 * tb : 0;
  f.lds = f.park_off + std::max(f.u_bytes, size_t(waves) * (tsh + dsh));
  return f.lds <= P->max_lds;
}

template <int PREC, typename T>
static const void* fused_kernel(int p, int len, int mode, int nw) {
#define STFD_FZ(PV, LV, MV, NV)                                  \
  if (p == PV && len == LV && mode == MV && nw == NV)           \
    return reinterpret_cast<const void*>(&fused_time_kernel<PREC, T, PV, LV, MV, NV>);
  STFD_FZ_INSTANCES
#undef STFD_FZ
  return nullptr;
}

// Tables of the fused form in its lane layout: block = column * waves + wave, slot m of a wave =
// mode wave * mpb + m of x_d in that column (spatial mode column + n_cols * m).
static int fused_tables(const HostProblem& hp, const FusedShape& f, TimeSolvePlan& tp) {
  const int n = hp.n_s[hp.d - 1];
  const int64_t ncols = hp.N_s / n;
  std::vector<int64_t> slots(size_t(ncols) * f.waves * f.mpb, -1);
  for (int64_t c = 0; c < ncols; ++c)
    for (int w = 0; w < f.waves; ++w)
      for (int ml = 0; ml < f.mpb; ++ml) {
        const int m = w * f.mpb + ml;
        if (m < n) slots[size_t((c * f.waves + w) * f.mpb + ml)] = c + ncols * m;
      }
  return f.mode == 2 ? time_solve_state_plan(hp, f.len, tp, &slots)
                     : time_solve_plan(hp, f.len, f.mode == 0, tp, &slots);
}

// Fused x_d products and time solves, in place allowed (in == out).
template <int PREC, typename T>
static int launch_fused_time(stfd_problem* P, const T* in, T* out, int64_t nrhs, const int* done, hipStream_t s) {
  const HostProblem& hp = P->hp;
  FusedShape f;
  if (!fused_shape(P, PREC, P->fz_len, P->fz_mode, P->fz_nw, f)) return STFD_EINVAL;
  if (nrhs < 1) return STFD_OK;
  if (nrhs > 65535) return STFD_EINVAL;
  const void* fn = fused_kernel<PREC, T>(hp.p_t, f.len, f.mode, f.nw);
  if (!fn) return STFD_EINVAL;
  const int l = hp.d - 1;
  FusedTimeArgs a;
  a.in = in;
  a.out = out;
  a.Uf = P->Upk_fwd[PREC][l];
  a.Ub = P->Upk_bwd[PREC][l];
  a.n = hp.n_s[l];
  a.n_t = hp.n_t;
  a.ld = f.ld;
  a.ks = mode_product_ks(PREC, a.n);
  a.segs = f.segs;
  a.mpb = f.mpb;
  a.n_cols = hp.N_s / a.n;
  a.u_bytes = f.u_bytes;
  a.park_off = f.park_off;
  a.done = done;
  if constexpr (std::is_same<T, double>::value) {
    a.Lf = P->FzL, a.Df = P->FzD, a.Tf = P->FzTf, a.Tb = P->FzTb, a.Sf = P->FzS, a.Hb = P->FzH, a.Mu = P->FzMu;
  } else {
    a.Lf = P->FzL32, a.Df = P->FzD32, a.Tf = P->FzTf32, a.Tb = P->FzTb32, a.Sf = P->FzS32, a.Hb = P->FzH32,
    a.Mu = P->FzMu32;
  }
  if ((f.mode == 2 && (!a.Sf || !a.Hb || !a.Mu)) || (f.mode < 2 && (!a.Lf || !a.Df)) ||
      (f.mode == 0 && (!a.Tf || !a.Tb)))
    return STFD_EINVAL;
  void* args[] = {&a};
  STFD_HIP(hipLaunchKernel(fn, dim3(unsigned(a.n_cols), unsigned(nrhs)), dim3(unsigned(f.waves * 64)), args,
                           f.lds, s));
  return STFD_OK;
}

// Algorithm 1 steps 2-4 on nrhs stacked vectors.  TW = storage of the intermediates that still
// have a physical direction; TY = storage of the mode-basis tensor that the time solves work on
// (written by the last forward product into the buffer that product does not read, and read by
// the first backward product).  FP64: both double; FP32 / BF16: both float.  (FP64 products with
// an FP32 mode-basis tensor and FP32 time solves were measured and dropped: they cost as many PCG
// iterations as FP32 products at a slower apply.)
// Timing events around one mode-product launch when stfd_timing_begin is active (pairs beyond the
// capacity are not recorded).
struct MpTimer {
  stfd_problem* P;
  hipStream_t s;
  bool on;
  MpTimer(stfd_problem* P_, hipStream_t s_) : P(P_), s(s_), on(P_->timing && P_->tev_used + 2 <= P_->tev.size()) {
    if (on) (void)hipEventRecord(P->tev[P->tev_used], s);
  }
  ~MpTimer() {
    if (on) {
      (void)hipEventRecord(P->tev[P->tev_used + 1], s);
      P->tev_used += 2;
    }
  }
};

template <int PREC, typename TW, typename TY>
static int apply_impl(stfd_problem* P, const double* r, double* s_out, int64_t nrhs, const int* done, hipStream_t s,
                      TW* w0, TW* w1, const DotEpilogue& ep) {
  const HostProblem& hp = P->hp;
  const int d = hp.d;
  // inner / outer sizes of each direction (reals)
  int64_t inner[3], outer[3], outer_rhs[3];
  int64_t below = 2 * int64_t(hp.n_t);
  for (int l = 0; l < d; ++l) {
    inner[l] = below;
    int64_t above = 1;
    for (int k = l + 1; k < d; ++k) above *= hp.n_s[k];
    outer_rhs[l] = above;
    outer[l] = above * nrhs;
    below *= hp.n_s[l];
  }
  // forward order of the directions (the backward products run in reverse): x_1 first on
  // the unit cube; on a mapped domain the per-mode direction x_1 must act on the modes of x_2,
  // so x_2 goes first
  int order[3] = {0, 1, 2};
  if (P->u_slice0)
    for (int k = 0; k < d; ++k) order[k] = d - 1 - k;
  auto slice = [&](int l) -> int64_t { return l == 0 ? P->upk_slice[PREC] : 0; };
  auto Ufwd = [&](int l) -> const void* { return P->Upk_fwd[PREC][l]; };
  auto Ubwd = [&](int l) -> const void* { return P->Upk_bwd[PREC][l]; };
  int rc;
  // the last direction fused with the time solves: x_1 .. x_{d-1} run as separate products
  static_assert(std::is_same<TW, TY>::value, "the fused form works in one storage type");
  const bool fused = P->fz_on && PREC != MP_BF16 && d >= 2 && !P->u_slice0;
  const int kf = fused ? d - 1 : d;  // directions with separate forward / backward products
  // step 2: y = (U_s^T (x) I) r; r (FP64) -> w0 -> w1 -> ... -> y (TY)
  void* bufs[2] = {w0, w1};
  int cur = 0;
  const void* src = r;  // input of the next product: r, then bufs[cur]
  for (int k = 0; k < kf; ++k) {
    const int l = order[k];
    void* dst = (k == 0) ? bufs[0] : bufs[cur ^ 1];
    const bool first = (k == 0), last = (k == d - 1);
    const MpTimer tm(P, s);
    if (first && last)
      rc = launch_mode_product<PREC, double, TY>(src, dst, Ufwd(l), hp.n_s[l], inner[l], outer[l], outer_rhs[l],
                                                 done, s, DotEpilogue(), slice(l), P->mp_rt[PREC][l]);
    else if (first)
      rc = launch_mode_product<PREC, double, TW>(src, dst, Ufwd(l), hp.n_s[l], inner[l], outer[l], outer_rhs[l],
                                                 done, s, DotEpilogue(), slice(l), P->mp_rt[PREC][l]);
    else if (last)
      rc = launch_mode_product<PREC, TW, TY>(src, dst, Ufwd(l), hp.n_s[l], inner[l], outer[l], outer_rhs[l], done,
                                             s, DotEpilogue(), slice(l), P->mp_rt[PREC][l]);
    else
      rc = launch_mode_product<PREC, TW, TW>(src, dst, Ufwd(l), hp.n_s[l], inner[l], outer[l], outer_rhs[l], done,
                                             s, DotEpilogue(), slice(l), P->mp_rt[PREC][l]);
    if (rc) return rc;
    if (k > 0) cur ^= 1;
    src = bufs[cur];
  }
  // step 3: N_s independent banded time solves, in place (fused: with the x_d products around
  // them, in place)
  if (fused) {
    if constexpr (PREC != MP_BF16)
      rc = launch_fused_time<PREC, TY>(P, static_cast<TY*>(bufs[cur]), static_cast<TY*>(bufs[cur]), nrhs, done, s);
  } else {
    rc = launch_time_solve<TY>(P, static_cast<TY*>(bufs[cur]), nrhs, done, s, static_cast<TY*>(bufs[cur ^ 1]));
  }
  if (rc) return rc;
  // step 4: s = (U_s (x) I) x in reverse order, the last product writes FP64 output
  for (int k = kf - 1; k >= 0; --k) {
    const int l = order[k];
    const bool first = (k == kf - 1), last = (k == 0);
    const MpTimer tm(P, s);
    if (last && first)
      return launch_mode_product<PREC, TY, double>(bufs[cur], s_out, Ubwd(l), hp.n_s[l], inner[l], outer[l],
                                                   outer_rhs[l], done, s, ep, slice(l), P->mp_rt[PREC][l]);
    if (last)
      return launch_mode_product<PREC, TW, double>(bufs[cur], s_out, Ubwd(l), hp.n_s[l], inner[l], outer[l],
                                                   outer_rhs[l], done, s, ep, slice(l), P->mp_rt[PREC][l]);
    if (first)
      rc = launch_mode_product<PREC, TY, TW>(bufs[cur], bufs[cur ^ 1], Ubwd(l), hp.n_s[l], inner[l], outer[l],
                                             outer_rhs[l], done, s, DotEpilogue(), slice(l), P->mp_rt[PREC][l]);
    else
      rc = launch_mode_product<PREC, TW, TW>(bufs[cur], bufs[cur ^ 1], Ubwd(l), hp.n_s[l], inner[l], outer[l],
                                             outer_rhs[l], done, s, DotEpilogue(), slice(l), P->mp_rt[PREC][l]);
    if (rc) return rc;
    cur ^= 1;
  }
  return STFD_OK;
}

// Algorithm 1 steps 2-4 with the intermediates in w0 / w1 (each 2 N nrhs reals of the working
// precision: doubles for FP64, floats otherwise)
static int apply_with_buffers(stfd_problem* P, const double* r, double* s_out, int64_t nrhs, int precision,
                              const int* done, hipStream_t s, void* w0, void* w1,
                              const DotEpilogue& ep = DotEpilogue()) {
  switch (precision) {
    case STFD_FP64:
      return apply_impl<MP_F64, double, double>(P, r, s_out, nrhs, done, s, static_cast<double*>(w0),
                                                static_cast<double*>(w1), ep);
    case STFD_FP32:
      return apply_impl<MP_F32, float, float>(P, r, s_out, nrhs, done, s, static_cast<float*>(w0),
                                              static_cast<float*>(w1), ep);
    case STFD_BF16:
      return apply_impl<MP_BF16, float, float>(P, r, s_out, nrhs, done, s, static_cast<float*>(w0),
                                               static_cast<float*>(w1), ep);
    default:
      return STFD_EINVAL;
  }
}

// bytes per real of the intermediates of an apply in this precision (the larger of the two kinds)
static size_t apply_elem_bytes(int precision) {
  return precision == STFD_FP64 ? sizeof(double) : sizeof(float);
}

static int apply_dispatch(stfd_problem* P, const double* r, double* s_out, int64_t nrhs, int precision,
                          const int* done, hipStream_t s, const DotEpilogue& ep = DotEpilogue()) {
  const bool f64 = apply_elem_bytes(precision) == sizeof(double);
  return apply_with_buffers(P, r, s_out, nrhs, precision, done, s, f64 ? (void*)P->work64[0] : (void*)P->work32[0],
                            f64 ? (void*)P->work64[1] : (void*)P->work32[1], ep);
}

// ---------------------------------------------------------------------------
// Setup-time autotuning (stfd_setup_desc.autotune): the launch shapes that have a choice are timed
// on the device on this problem's own sizes and the fastest is kept.
//  * mode products: one or two 16-row groups per wave, or the wide form (every column group per
//    wave), for n <= 80, per direction and precision;
//  * time solve: segment length (every compiled one with at most 64 segments) x transfers read
//    from tables or computed in the solve, where the tables of every candidate are cheap to build
//    (N_s n_t <= kTuneTsRows); larger problems try the segment lengths of the factor-in-kernel
//    form only (its tables are P^2 values per segment).
// Each candidate runs 2 untimed and 5 timed launches on a private stream; the median decides.
// ---------------------------------------------------------------------------
constexpr int64_t kTuneTsRows = int64_t(1) << 21;

struct TuneClock {
  hipStream_t s = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  ~TuneClock() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (s) (void)hipStreamDestroy(s);
  }
  int init() {
    STFD_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    STFD_HIP(hipEventCreate(&a));
    STFD_HIP(hipEventCreate(&b));
    return STFD_OK;
  }
  // median time (ms) of 5 launches after 2 untimed ones
  template <typename F>
  int median(F launch, float* ms) {
    for (int w = 0; w < 2; ++w)
      if (int rc = launch()) return rc;
    float t[5];
    for (int r = 0; r < 5; ++r) {
      STFD_HIP(hipEventRecord(a, s));
      if (int rc = launch()) return rc;
      STFD_HIP(hipEventRecord(b, s));
      STFD_HIP(hipEventSynchronize(b));
      STFD_HIP(hipEventElapsedTime(&t[r], a, b));
    }
    std::sort(t, t + 5);
    *ms = t[2];
    return STFD_OK;
  }
};

// Row groups of every mode product (forward operand, one right-hand side, FP64 in FP64 out or
// FP32 in FP32 out as inside the applies); x, y: device buffers of 2 N doubles.
static int tune_mode_products(stfd_problem* P, TuneClock& C, void* x, void* y) {
  const HostProblem& hp = P->hp;
  for (int prec = MP_F64; prec <= MP_BF16; ++prec)
    for (int l = 0; l < hp.d; ++l) {
      const int n = hp.n_s[l];
      if (n > 80) continue;  // one row group only
      const int64_t inner = mp_inner(hp, l), outer = mp_outer(hp, l);
      const int64_t slice = l == 0 ? P->upk_slice[prec] : 0;
      const void* U = P->Upk_fwd[prec][l];
      float best = 0.0f;
      int best_rt = P->mp_rt[prec][l];
      for (int rt = 1; rt <= kMpWide; ++rt) {
        if (rt == kMpWide && slice != 0) continue;  // the wide form takes one operand
        auto launch = [&]() -> int {
          if (prec == MP_F64)
            return launch_mode_product<MP_F64, double, double>(x, y, U, n, inner, outer, outer, nullptr, C.s,
                                                               DotEpilogue(), slice, rt);
          if (prec == MP_F32)
            return launch_mode_product<MP_F32, float, float>(x, y, U, n, inner, outer, outer, nullptr, C.s,
                                                             DotEpilogue(), slice, rt);
          return launch_mode_product<MP_BF16, float, float>(x, y, U, n, inner, outer, outer, nullptr, C.s,
                                                            DotEpilogue(), slice, rt);
        };
        float ms = 0.0f;
        if (int rc = C.median(launch, &ms)) return rc;
        if (rt == 1 || ms < best) {
          best = ms;
          best_rt = rt;
        }
      }
      P->mp_rt[prec][l] = best_rt;
    }
  set_last_blocks(P);
  return STFD_OK;
}

// Host tables of the time solve for segment length len and form mode (0: L, 1/D and transfers;
// 1: L and 1/D; 2: entry states, time bands and nu lambda_i).
static int time_tables(const HostProblem& hp, int len, int mode, TimeSolvePlan& tp) {
  return mode == 2 ? time_solve_state_plan(hp, len, tp) : time_solve_plan(hp, len, mode == 0, tp);
}

// Segment length and form of the FP64 time solve (sets P->ts_len and P->ts_mode).
static int tune_time_solve(stfd_problem* P, TuneClock& C) {
  const HostProblem& hp = P->hp;
  int cand[4];
  const int nc = time_segment_candidates(hp.n_t, hp.p_t, cand);
  double* y = nullptr;
  STFD_HIP(hipMalloc(&y, sizeof(double) * 2 * size_t(hp.N)));
  STFD_HIP(hipMemsetAsync(y, 0, sizeof(double) * 2 * size_t(hp.N), C.s));
  float best = 0.0f;
  int best_len = P->ts_len, rc = STFD_OK;
  int best_mode = P->ts_mode;
  bool have = false;
  for (int c = 0; c < nc && rc == STFD_OK; ++c)
    for (int mode = 0; mode < 3 && rc == STFD_OK; ++mode) {
      if (mode < 2 && hp.N_s * hp.n_t > kTuneTsRows) continue;  // full tables: large grids skip them
      TimeSolvePlan tp;
      if (time_tables(hp, cand[c], mode, tp) != 0) continue;
      double* buf[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
      const std::vector<double>* src[7] = {&tp.Lf, &tp.Df, &tp.Tf, &tp.Tb, &tp.Sf, &tp.Hb, &tp.mu};
      for (int k = 0; k < 7 && rc == STFD_OK; ++k) {
        if (src[k]->empty()) continue;
        hipError_t e = hipMalloc(&buf[k], sizeof(double) * src[k]->size());
        if (e == hipSuccess) e = hipMemcpy(buf[k], src[k]->data(), sizeof(double) * src[k]->size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
          g_last_hip_error = int(e);
          rc = STFD_EHIP;
        }
      }
      if (rc == STFD_OK) {
        P->TsL = buf[0];
        P->TsD = buf[1];
        P->TsTf = buf[2];
        P->TsTb = buf[3];
        P->TsS = buf[4];
        P->TsH = buf[5];
        P->TsMu = buf[6];
        P->ts_mode = mode;
        P->ts_len = tp.len;
        P->ts_segs = tp.segs;
        P->ts_mpb = tp.mpb;
        P->ts_blocks = tp.blocks;
        float ms = 0.0f;
        rc = C.median([&]() { return launch_time_solve<double>(P, y, 1, nullptr, C.s, nullptr); }, &ms);
        if (rc == STFD_OK && (!have || ms < best)) {
          have = true;
          best = ms;
          best_len = tp.len;
          best_mode = mode;
        }
      }
      (void)hipStreamSynchronize(C.s);
      for (double* b : buf)
        if (b) (void)hipFree(b);
      P->TsL = P->TsD = P->TsTf = P->TsTb = P->TsS = P->TsH = P->TsMu = nullptr;
    }
  (void)hipFree(y);
  if (rc != STFD_OK) return rc;
  P->ts_len = best_len;
  P->ts_mode = best_mode;
  return STFD_OK;
}

// Fused form: the compiled candidates that fit this problem (FP64 shape), in the order of the
// default choice: the time-solve form the grid calls for (factor in kernel for more columns than
// 4 blocks per CU, else tables), then four-wave blocks, then the longer segment.
static std::vector<FusedShape> fused_candidates(const stfd_problem* P) {
  std::vector<FusedShape> c;
  FusedShape f, f32;
#define STFD_FZ(PV, LV, MV, NV)                                                                   \
  if (P->hp.p_t == PV && fused_shape(P, MP_F64, LV, MV, NV, f) && fused_shape(P, MP_F32, LV, MV, NV, f32)) \
    c.push_back(f);
  STFD_FZ_INSTANCES
#undef STFD_FZ
  if (c.empty()) return c;
  const int64_t ncols = P->hp.N_s / P->hp.n_s[P->hp.d - 1];
  const int want = ncols > 4 * int64_t(P->n_cus) ? 2 : 0;
  std::stable_sort(c.begin(), c.end(), [&](const FusedShape& x, const FusedShape& y) {
    if ((x.mode == want) != (y.mode == want)) return x.mode == want;
    if (x.nw != y.nw) return x.nw < y.nw;
    return x.len > y.len;
  });
  return c;
}

// Device tables of the fused form f (FP64 and FP32 copies).  keep: handle-owned (freed with the
// handle); else plain allocations the caller frees with fused_free.
static int fused_upload(stfd_problem* P, const FusedShape& f, bool keep) {
  TimeSolvePlan tp;
  if (fused_tables(P->hp, f, tp) != 0) return STFD_EINVAL;
  const std::vector<double>* src[7] = {&tp.Lf, &tp.Df, &tp.Tf, &tp.Tb, &tp.Sf, &tp.Hb, &tp.mu};
  double** d64[7] = {&P->FzL, &P->FzD, &P->FzTf, &P->FzTb, &P->FzS, &P->FzH, &P->FzMu};
  float** d32[7] = {&P->FzL32, &P->FzD32, &P->FzTf32, &P->FzTb32, &P->FzS32, &P->FzH32, &P->FzMu32};
  for (int k = 0; k < 7; ++k) {
    *d64[k] = nullptr;
    *d32[k] = nullptr;
  }
  for (int k = 0; k < 7; ++k) {
    if (src[k]->empty()) continue;
    const std::vector<float> v32(src[k]->begin(), src[k]->end());
    int rc;
    if (keep) {
      if ((rc = upload(P, d64[k], src[k]->data(), src[k]->size())) || (rc = upload(P, d32[k], v32.data(), v32.size())))
        return rc;
    } else {
      hipError_t e = hipMalloc(d64[k], sizeof(double) * src[k]->size());
      if (e == hipSuccess) e = hipMalloc(d32[k], sizeof(float) * v32.size());
      if (e == hipSuccess)
        e = hipMemcpy(*d64[k], src[k]->data(), sizeof(double) * src[k]->size(), hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(*d32[k], v32.data(), sizeof(float) * v32.size(), hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        g_last_hip_error = int(e);
        return STFD_EHIP;
      }
    }
  }
  P->fz_len = f.len;
  P->fz_mode = f.mode;
  P->fz_nw = f.nw;
  P->fz_waves = f.waves;
  P->fz_segs = f.segs;
  P->fz_mpb = f.mpb;
  return STFD_OK;
}
static void fused_free(stfd_problem* P) {
  void* p[14] = {P->FzL, P->FzD, P->FzTf, P->FzTb, P->FzS, P->FzH, P->FzMu,
                 P->FzL32, P->FzD32, P->FzTf32, P->FzTb32, P->FzS32, P->FzH32, P->FzMu32};
  for (void* q : p)
    if (q) (void)hipFree(q);
  P->FzL = P->FzD = P->FzTf = P->FzTb = P->FzS = P->FzH = P->FzMu = nullptr;
  P->FzL32 = P->FzD32 = P->FzTf32 = P->FzTb32 = P->FzS32 = P->FzH32 = P->FzMu32 = nullptr;
  P->fz_len = 0;
}
// LDS beyond the default per-block limit is granted per kernel
static int fused_allow_lds(const stfd_problem* P, const FusedShape& f) {
  const void* k64 = fused_kernel<MP_F64, double>(P->hp.p_t, f.len, f.mode, f.nw);
  const void* k32 = fused_kernel<MP_F32, float>(P->hp.p_t, f.len, f.mode, f.nw);
  if (!k64 || !k32) return STFD_EINVAL;
  STFD_HIP(hipFuncSetAttribute(k64, hipFuncAttributeMaxDynamicSharedMemorySize, int(f.lds)));
  FusedShape f32;
  if (!fused_shape(P, MP_F32, f.len, f.mode, f.nw, f32)) return STFD_EINVAL;
  STFD_HIP(hipFuncSetAttribute(k32, hipFuncAttributeMaxDynamicSharedMemorySize, int(f32.lds)));
  return STFD_OK;
}

// Fused form at setup: tables of the chosen candidate; with the autotune, every candidate and the
// separate launches are timed as whole FP64 applies (x, y: 2 N doubles) and the fastest is kept,
// else the first candidate is built and left off: on the 3D workloads the fused launch takes
// longer than the three it replaces (one block per CU, whose latency-bound time solves no other
// block's products overlap), so the heuristic keeps the separate launches.
static int setup_fused(stfd_problem* P, int want_len, bool autotune, TuneClock* C, double* x, double* y) {
  std::vector<FusedShape> cand = fused_candidates(P);
  P->fz_on = false;
  if (want_len > 0) {
    cand.erase(std::remove_if(cand.begin(), cand.end(), [&](const FusedShape& f) { return f.len != want_len; }),
               cand.end());
    if (cand.empty()) return STFD_EINVAL;
  }
  if (cand.empty()) return STFD_OK;
  int rc;
  size_t pick = 0;
  bool on = false;
  if (autotune) {
    auto apply = [&]() { return apply_dispatch(P, x, y, 1, STFD_FP64, nullptr, C->s); };
    float best = 0.0f;
    if ((rc = C->median(apply, &best))) return rc;  // separate launches
    on = false;
    for (size_t k = 0; k < cand.size(); ++k) {
      if ((rc = fused_allow_lds(P, cand[k]))) return rc;
      rc = fused_upload(P, cand[k], false);
      float ms = 0.0f;
      if (rc == STFD_OK) {
        P->fz_on = true;
        rc = C->median(apply, &ms);
        P->fz_on = false;
      }
      (void)hipStreamSynchronize(C->s);
      fused_free(P);
      if (rc) return rc;
      if (ms < best) {
        best = ms;
        pick = k;
        on = true;
      }
    }
  }
  if ((rc = fused_allow_lds(P, cand[pick])) || (rc = fused_upload(P, cand[pick], true))) return rc;
  P->fz_on = on;
  return STFD_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free apply (stfd_apply_preconditioner_static): the two intermediate
// tensors of Algorithm 1 steps 2-4 live in a file-scope device array of fixed size instead of the
// handle's work buffers.  Host code never passes the array's name to a kernel (on the host it is
// a stand-in, not a device address): its device address is taken once per device with
// hipGetSymbolAddress and kept in g_scratch_dev.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device, two halves of 32 MiB
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];
static void* g_scratch_dev[kMaxDevices] = {};
static std::mutex g_scratch_mutex;

// Device address of `scratch` on the current device (looked up on the first use per device).
static int scratch_address(void** out) {
  int dev = 0;
  STFD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return STFD_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    STFD_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return STFD_EHIP;
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return STFD_OK;
}

constexpr int kMvRowBatch = 1;  // stencil rows whose loads are issued together (measured best)

// spatial points per matvec block: whole points, at most kMvLanes lanes, coefficients (or Z) in
// kMvLds.  Between half that cap and the cap, K minimises the points of the busiest compute unit,
// ceil(blocks / CUs) K (ties: the larger K, fewer blocks): every block is resident from the start,
// the kernel ends with its slowest CU, and a CU holding one block more than the others sets the
// end (with 7-point blocks of the 65^2 x 66 grid, 604 blocks leave 92 CUs with three blocks;
// 6-point blocks cap every CU at 18 points instead of 21, measured 16.4 -> 15.5 us).  Smaller
// blocks would pay the staging of the time bands too often.
static int matvec_points_per_block(const HostProblem& hp, int n_cus) {
  const size_t per_point = std::max<size_t>(size_t(hp.stencil) * 3, size_t(hp.n_t) * 6) * sizeof(double);
  const int kmax = std::max(1, std::min<int>(kMvLanes / hp.n_t, int(kMvLds / per_point)));
  int best = kmax;
  int64_t best_load = INT64_MAX;
  for (int K = kmax; K >= (kmax + 1) / 2; --K) {
    const int64_t blocks = (hp.N_s + K - 1) / K;
    const int64_t load = (blocks + n_cus - 1) / n_cus * K;
    if (load < best_load) {
      best_load = load;
      best = K;
    }
  }
  return best;
}

static int matvec_dispatch(stfd_problem* P, const double* x, double* y, int64_t nrhs, double* partial,
                           const int* done, hipStream_t s) {
  if (P->sf_on) {
    const int he = sumfac_matvec(P->sf, x, y, nrhs, partial, done, s);
    if (he != 0) {
      g_last_hip_error = he;
      return STFD_EHIP;
    }
    return STFD_OK;
  }
  const HostProblem& hp = P->hp;
  if (P->mv_long) {
    if (nrhs < 1) return STFD_OK;
    hipLaunchKernelGGL(matvec_long1d_kernel, dim3(unsigned(P->mv_blocks), unsigned(nrhs)), dim3(kMvLongBlock), 0, s,
                       x, y, P->Sc, P->TbL, hp.n_t, hp.p_t, hp.n_s[0], hp.p_s, P->mv_blocks, partial, done);
    STFD_HIP(hipGetLastError());
    return STFD_OK;
  }
  MatvecArgs a;
  a.x = x;
  a.y = y;
  a.Sc = P->Sc;
  a.TbL = P->TbL;
  a.n_t = hp.n_t;
  a.pt = hp.p_t;
  a.n1 = hp.n_s[0];
  a.n2 = hp.n_s[1];
  a.n3 = hp.n_s[2];
  a.K = P->mv_points;
  a.N_s = hp.N_s;
  a.blocks_per_rhs = P->mv_blocks;
  a.nrhs = nrhs;
  a.xcd_span = (P->mv_blocks * nrhs + kXcds - 1) / kXcds;
  a.partial = partial;
  a.done = done;
  const int st = hp.stencil, wt = 2 * hp.p_t + 1;
  const size_t area = (std::max<size_t>(size_t(a.K) * st * 3, size_t(a.K) * hp.n_t * 6) + 1) / 2 * 2;
  const size_t lds = (area + size_t(hp.n_t) * wt * 4) * sizeof(double);
  const int lanes = (a.K * hp.n_t + 63) / 64 * 64;
  const dim3 grid(static_cast<unsigned>(a.xcd_span * kXcds)), block(static_cast<unsigned>(lanes));
#define STFD_MV_T(DV, PV, TV)                                                                     \
  case TV:                                                                                       \
    hipLaunchKernelGGL((matvec_kernel<DV, PV, TV, kMvRowBatch>), grid, block, lds, s, a);         \
    break;
#define STFD_MV(DV, PV)                                                                           \
  if (hp.d == DV && hp.p_s == PV) {                                                              \
    switch (hp.p_t) {                                                                            \
      STFD_MV_T(DV, PV, 1) STFD_MV_T(DV, PV, 2) STFD_MV_T(DV, PV, 3) STFD_MV_T(DV, PV, 4)         \
      STFD_MV_T(DV, PV, 5) STFD_MV_T(DV, PV, 6)                                                  \
      default:                                                                                   \
        return STFD_EINVAL;                                                                      \
    }                                                                                            \
    STFD_HIP(hipGetLastError());                                                                 \
    return STFD_OK;                                                                              \
  }
  STFD_MV(1, 2) STFD_MV(1, 3) STFD_MV(1, 4) STFD_MV(1, 5) STFD_MV(1, 6)
  STFD_MV(2, 2) STFD_MV(2, 3) STFD_MV(2, 4) STFD_MV(2, 5)
  STFD_MV(3, 2) STFD_MV(3, 3) STFD_MV(3, 4)
#undef STFD_MV
#undef STFD_MV_T
  return STFD_EINVAL;
}

}  // namespace stfd

using namespace stfd;

extern "C" {

const char* stfd_strerror(int code) {
  switch (code) {
    case STFD_OK: return "ok";
    case STFD_NOT_CONVERGED: return "PCG did not converge within maxit iterations";
    case STFD_EINVAL: return "invalid argument";
    case STFD_ENOTSPD: return "matrix not (Hermitian) positive definite";
    case STFD_EBREAKDOWN: return "PCG breakdown (non-finite value or non-positive curvature)";
    case STFD_ENOMEM: return "allocation failed";
    case STFD_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

int stfd_last_hip_error(void) { return g_last_hip_error; }

int stfd_quad_points(const double* knots, int n_knots, int degree, int n_quad, double scale, double* pts,
                     double* wts, int* n_out) {
  if (!n_out || degree < 1 || n_quad < 0 || !(scale > 0.0)) return STFD_EINVAL;
  if (validate_knots(knots, n_knots, degree, degree)) return STFD_EINVAL;
  Direction D;
  if (build_direction(knots, n_knots, degree, n_quad ? n_quad : degree + 1, scale, D)) return STFD_EINVAL;
  *n_out = int(D.x.size());
  if (pts) std::memcpy(pts, D.x.data(), D.x.size() * sizeof(double));
  if (wts) std::memcpy(wts, D.w.data(), D.w.size() * sizeof(double));
  return STFD_OK;
}

namespace stfd {

// Point the load-vector plan at the device copies of the current model's arrays.
static void set_plan_model(stfd_problem* P) {
  const SpatialModel& m = P->model;
  LoadPlan& L = P->load;
  auto arr = [&](int k) -> const double* { return k >= 0 ? P->sdev.arrays[size_t(k)] : nullptr; };
  L.Vq = arr(m.V);
  L.Jq = arr(m.J);
  L.n_lap = int(std::min<size_t>(m.lap.size(), 4));
  for (int k = 0; k < L.n_lap; ++k) {
    for (int l = 0; l < 3; ++l) L.lap_ord[k][l] = m.lap[size_t(k)].ord[l];
    L.lap_c[k] = arr(m.lap[size_t(k)].coef);
    L.lap_cJ[k] = arr(m.lap[size_t(k)].coefJ);
  }
}

}  // namespace stfd

int stfd_update_potential(stfd_problem* P, const double* V_quad, void* stream) {
  if (!P) return STFD_EINVAL;
  stfd::graph_cache_clear(P);
  hipStream_t s = static_cast<hipStream_t>(stream);
  SpatialModel m;
  if (build_spatial_model(P->hp, P->geom, V_quad, m)) return STFD_EINVAL;
  std::vector<double> bands[3];
  if (P->sf_on) {
    // the sum-factorised matvec needs V as a sum of 1D functions
    if (sumfac_bands(P->hp, V_quad, bands)) return STFD_EINVAL;
    STFD_HIP(hipStreamSynchronize(s));
    for (int l = 0; l < P->hp.d; ++l)
      STFD_HIP(hipMemcpy(P->sf.bands[l], bands[l].data(), bands[l].size() * sizeof(double), hipMemcpyHostToDevice));
  }
  P->model = std::move(m);
  int he = spatial_device_apply(P->hp, P->model, P->sdev, P->sf_on ? nullptr : P->Sc, s);
  if (he == 0) he = int(hipStreamSynchronize(s));
  stfd::set_plan_model(P);
  if (he != 0) {
    g_last_hip_error = he;
    return STFD_EHIP;
  }
  return STFD_OK;
}

int stfd_map_points(const stfd_problem* P, const double* xi, int64_t n, double* x) {
  if (!P || n < 0 || (n > 0 && (!xi || !x))) return STFD_EINVAL;
  map_points(P->geom, P->hp.d, xi, n, x);
  return STFD_OK;
}

void stfd_destroy(stfd_problem* P) {
  if (!P) return;
  stfd::graph_cache_clear(P);
  for (hipEvent_t e : P->tev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : P->job_ev)
    if (e) (void)hipEventDestroy(e);
  if (P->job_stream) (void)hipStreamDestroy(P->job_stream);
  for (void* p : P->allocs) (void)hipFree(p);
  stfd::load_plan_free(P->load);
  stfd::spatial_device_free(P->sdev);
  if (P->sc_host) (void)hipHostFree(P->sc_host);
  if (P->lift_status_host) (void)hipHostFree(P->lift_status_host);
  delete P;
}

int stfd_setup(const stfd_setup_desc* desc, stfd_problem** out) {
  if (!desc || !out) return STFD_EINVAL;
  *out = nullptr;
  if (desc->max_nrhs < 1 || desc->d < 1 || desc->d > 3) return STFD_EINVAL;
  stfd_setup_desc_view v;
  v.d = desc->d;
  v.p_t = desc->p_t;
  v.p_s = desc->p_s;
  v.knots_t = desc->knots_t;
  v.n_knots_t = desc->n_knots_t;
  for (int l = 0; l < 3; ++l) {
    v.knots_s[l] = desc->knots_s[l];
    v.n_knots_s[l] = desc->n_knots_s[l];
  }
  v.T = desc->T;
  v.nu = desc->nu;
  v.n_quad = desc->n_quad;
  Geometry geom;
  geom.kind = desc->geometry;
  geom.r0 = desc->geom[0];
  geom.r1 = desc->geom[1];
  if (geom.kind != GEOM_UNIT && !(geom.kind == GEOM_QUARTER_ANNULUS && desc->d == 2 && geom.r0 > 0.0 &&
                                   geom.r1 > geom.r0 && std::isfinite(geom.r1)))
    return STFD_EINVAL;
  v.kronecker_base = (geom.kind == GEOM_UNIT);
  v.stencils = false;  // built below unless the matvec runs sum-factorised
  if (desc->matvec < STFD_MATVEC_AUTO || desc->matvec > STFD_MATVEC_SUMFAC) return STFD_EINVAL;
  if (desc->time_condition != STFD_TIME_INITIAL && desc->time_condition != STFD_TIME_FINAL) return STFD_EINVAL;
  if (desc->autotune != 0 && desc->autotune != 1) return STFD_EINVAL;
  if (desc->precond_shift != STFD_SHIFT_NONE && desc->precond_shift != STFD_SHIFT_MEAN_POTENTIAL) return STFD_EINVAL;
  if (desc->precond_shift == STFD_SHIFT_MEAN_POTENTIAL && geom.kind != GEOM_UNIT) return STFD_EINVAL;
  if (desc->fused_segment_length < 0) return STFD_EINVAL;
  if (desc->time_condition == STFD_TIME_FINAL && geom.kind != GEOM_UNIT) return STFD_EINVAL;
  v.time_final = desc->time_condition == STFD_TIME_FINAL;
  // sizes from the knot counts (m = knots - degree - 1 functions; the reduced bases drop two in
  // space and one in time), checked before the host setup spends time on them
  {
    const int64_t n_t = int64_t(desc->n_knots_t) - desc->p_t - 2;
    const bool one_d = desc->d == 1;
    if (n_t > (one_d ? kLongMaxNt : kMvMaxNt)) return STFD_EINVAL;
    for (int l = 0; l < desc->d; ++l)
      if (int64_t(desc->n_knots_s[l]) - desc->p_s - 3 > (one_d ? kLongMaxN : kMaxModeN)) return STFD_EINVAL;
  }
  stfd_problem* P = new (std::nothrow) stfd_problem;
  if (!P) return STFD_ENOMEM;
  int rc = host_setup(v, P->hp);
  if (rc == 0) {
    const HostProblem& hp = P->hp;
    const bool long1d = hp.d == 1 && hp.n_s[0] <= kLongMaxN && hp.n_t <= kLongMaxNt;
    for (int l = 0; l < hp.d; ++l)
      if (hp.n_s[l] > kMaxModeN && !long1d) rc = -1;
    if (hp.p_t > 6) rc = -1;
    bool mv_ok = (hp.d == 1 && hp.p_s <= 6) || (hp.d == 2 && hp.p_s <= 5) || (hp.d == 3 && hp.p_s <= 4);
    if (!mv_ok) rc = -1;
    if (hp.n_t > kMvMaxNt && !long1d) rc = -1;
  }
  if (rc) {
    delete P;
    return rc;
  }
  const HostProblem& hp = P->hp;
  P->geom = geom;
  if (build_spatial_model(hp, geom, desc->V_quad, P->model)) {
    delete P;
    return STFD_EINVAL;
  }
  // preconditioner shifted by the mean potential: the time pencils H_i are refactorised with
  // mu_i = nu lambda_i + c
  if (desc->precond_shift == STFD_SHIFT_MEAN_POTENTIAL && desc->V_quad) {
    P->hp.shift = mean_potential(hp, desc->V_quad);
    if (time_factors(P->hp) != 0) {
      delete P;
      return STFD_ENOTSPD;
    }
  }
  // matvec form: sum-factorised on the unit cube in 3D (by default) when V is a sum of 1D functions
  std::vector<double> sf_bands[3];
  {
    const bool want = desc->matvec == STFD_MATVEC_SUMFAC || (desc->matvec == STFD_MATVEC_AUTO && hp.d == 3);
    const bool able = geom.kind == GEOM_UNIT && hp.d >= 2 && hp.p_s <= 5 && sumfac_bands(hp, desc->V_quad, sf_bands) == 0;
    if (desc->matvec == STFD_MATVEC_SUMFAC && !able) {
      delete P;
      return STFD_EINVAL;
    }
    P->sf_on = want && able;
    if (!P->sf_on) base_stencils(P->hp, v.kronecker_base);
  }
  P->max_nrhs = desc->max_nrhs;
  P->n2 = 2 * hp.N;
  // on the quarter annulus P-hat uses the physical mass and stiffness matrices (two-level
  // pencils) unless the parametric one is requested
  if (geom.kind == GEOM_QUARTER_ANNULUS && desc->precond == STFD_PRECOND_AUTO) {
    const int gp = geometry_pencils(P->hp, geom);
    if (gp) {
      delete P;
      return gp == -2 ? STFD_ENOTSPD : STFD_EINVAL;
    }
  }
  // pencils: forward operand U, backward operand U^T (direction 0 of a mapped domain: one
  // matrix per mode of direction 1)
  for (int l = 0; l < hp.d; ++l) {
    const int n = hp.n_s[l];
    const bool sliced = (l == 0 && !hp.Uslice.empty());
    const std::vector<double>& Uf = sliced ? hp.Uslice : hp.U[l];
    const int nsl = sliced ? hp.n_s[1] : 1;
    std::vector<double> Ut(Uf.size());
    for (int k = 0; k < nsl; ++k)
      for (int j = 0; j < n; ++j)
        for (int a = 0; a < n; ++a)
          Ut[(size_t(k) * n + j) * n + a] = Uf[(size_t(k) * n + a) * n + j];
    for (int prec = MP_F64; prec <= MP_BF16; ++prec) {
      const int K = prec == MP_BF16 ? 16 : 4, E = K / 4, KS = mode_product_ks(prec, n);
      if (prec == MP_F64) {
        std::vector<double> pf, pb;
        pack_mode_operand(Uf.data(), n, nsl, K, E, KS, pf);
        pack_mode_operand(Ut.data(), n, nsl, K, E, KS, pb);
        rc = upload(P, reinterpret_cast<double**>(&P->Upk_fwd[prec][l]), pf.data(), pf.size());
        if (!rc) rc = upload(P, reinterpret_cast<double**>(&P->Upk_bwd[prec][l]), pb.data(), pb.size());
      } else {
        std::vector<float> pf, pb;
        pack_mode_operand(Uf.data(), n, nsl, K, E, KS, pf);
        pack_mode_operand(Ut.data(), n, nsl, K, E, KS, pb);
        rc = upload(P, reinterpret_cast<float**>(&P->Upk_fwd[prec][l]), pf.data(), pf.size());
        if (!rc) rc = upload(P, reinterpret_cast<float**>(&P->Upk_bwd[prec][l]), pb.data(), pb.size());
      }
      if (rc) {
        stfd_destroy(P);
        return rc;
      }
      if (sliced) P->upk_slice[prec] = int64_t((n + 15) / 16) * KS * 64 * E;
    }
    if (sliced) P->u_slice0 = int64_t(n) * n;
  }
  {
    int dev = 0, lds = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
      P->max_lds = size_t(lds);
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      P->n_cus = cus;
    P->ts_len = time_segment_length(hp.n_t, hp.p_t);
    P->mv_long = hp.d == 1 && hp.n_t > kMvMaxNt;
    if ((P->ts_len == 0 && hp.d != 1) || (hp.n_t > kMvMaxNt && !P->mv_long) ||
        hp.N_s * hp.n_t * 16 >= int64_t(kMvBadOffset)) {
      stfd_destroy(P);
      return STFD_EINVAL;
    }
  }
  // segmented time-solve tables, time bands, spatial coefficients
  {
    TimeSolvePlan tp;
    // all tables where one right-hand side's grid holds at most one wave per SIMD (the solve is
    // bound by its dependent chain), else the factor-in-kernel form (bound by table traffic)
    if (P->ts_len == 0) {
      P->ts_mode = 3;  // no segmented layout holds the axis: one lane per mode
    } else {
      const int mpb = 64 / ((hp.n_t + P->ts_len - 1) / P->ts_len);  // modes per block
      P->ts_mode = (hp.N_s + mpb - 1) / mpb <= 4 * int64_t(P->n_cus) ? 0 : 2;
    }
    if (desc->autotune) {
      const auto t0 = std::chrono::steady_clock::now();
      TuneClock C;
      if ((rc = C.init()) || (rc = tune_time_solve(P, C))) {
        stfd_destroy(P);
        return rc;
      }
      P->tune_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      P->autotuned = true;
    }
    if (P->ts_mode == 3) {
      // the host factors as they are: Lfac[t][k-1][mode] (complex) and 1/D[t][mode]
      tp.Lf.resize(hp.Lfac.size() * 2);
      for (size_t k = 0; k < hp.Lfac.size(); ++k) {
        tp.Lf[2 * k] = hp.Lfac[k].real();
        tp.Lf[2 * k + 1] = hp.Lfac[k].imag();
      }
      tp.Df = hp.Dinv;
    } else if (time_tables(hp, P->ts_len, P->ts_mode, tp) != 0) {
      stfd_destroy(P);
      return STFD_EINVAL;
    }
    P->ts_segs = tp.segs;
    P->ts_mpb = tp.mpb;
    P->ts_blocks = tp.blocks;
    // FP64 tables and FP32 copies (time solves of the FP32 / BF16 applies); empty ones stay null
    auto f32 = [](const std::vector<double>& v) { return std::vector<float>(v.begin(), v.end()); };
    const std::vector<double>* src[7] = {&tp.Lf, &tp.Df, &tp.Tf, &tp.Tb, &tp.Sf, &tp.Hb, &tp.mu};
    double** d64[7] = {&P->TsL, &P->TsD, &P->TsTf, &P->TsTb, &P->TsS, &P->TsH, &P->TsMu};
    float** d32[7] = {&P->TsL32, &P->TsD32, &P->TsTf32, &P->TsTb32, &P->TsS32, &P->TsH32, &P->TsMu32};
    for (int k = 0; k < 7; ++k) {
      if (src[k]->empty()) continue;
      const std::vector<float> v32 = f32(*src[k]);
      if ((rc = upload(P, d64[k], src[k]->data(), src[k]->size())) || (rc = upload(P, d32[k], v32.data(), v32.size()))) {
        stfd_destroy(P);
        return rc;
      }
    }
    // spatial coefficients interleaved per row and stencil offset: [N_s][stencil][3];
    // V-free unit-cube base from the host, weighted terms (potential, geometry) added on the device
    // (no stencils are stored for the sum-factorised matvec: hp.Sc is empty then)
    std::vector<double> ScI(hp.Sc.size());
    const size_t ns = hp.Sc.size() / 3;
    for (size_t is = 0; is < ns; ++is)
      for (int k = 0; k < 3; ++k) ScI[is * 3 + k] = hp.Sc[k * ns + is];
    // time bands in the matvec's LDS layout [t][dt][4] = (L_t, M_t, K_t, 0), zero where t + dt - p_t
    // falls outside the time axis
    const int wtb = 2 * hp.p_t + 1;
    std::vector<double> TbL(size_t(hp.n_t) * wtb * 4, 0.0);
    for (int k = 0; k < 3; ++k)
      for (int t = 0; t < hp.n_t; ++t)
        for (int dt = 0; dt < wtb; ++dt) {
          const int tt = t + dt - hp.p_t;
          if (tt >= 0 && tt < hp.n_t)
            TbL[(size_t(t) * wtb + dt) * 4 + k] = hp.Tband[(size_t(k) * hp.n_t + t) * wtb + dt];
        }
    if ((rc = upload(P, &P->TbL, TbL.data(), TbL.size())) ||
        (!P->sf_on && (rc = dev_alloc(P, &P->Sc, ScI.size())))) {
      stfd_destroy(P);
      return rc;
    }
    int he = spatial_device_init(hp, (P->model.kronecker_base && !P->sf_on) ? ScI.data() : nullptr, P->sdev);
    if (he == 0) he = spatial_device_apply(hp, P->model, P->sdev, P->sf_on ? nullptr : P->Sc, nullptr);
    if (he == 0) he = int(hipDeviceSynchronize());
    if (he != 0) {
      g_last_hip_error = he;
      stfd_destroy(P);
      return STFD_EHIP;
    }
  }
  const size_t nvec = size_t(P->n2) * P->max_nrhs;
  for (int k = 0; k < 2; ++k)
    if ((rc = dev_alloc(P, &P->work64[k], nvec)) || (rc = dev_alloc(P, &P->work32[k], nvec))) {
      stfd_destroy(P);
      return rc;
    }
  for (int k = 0; k < 5; ++k)
    if ((rc = dev_alloc(P, &P->vec[k], nvec))) {
      stfd_destroy(P);
      return rc;
    }
  // matvec launch shape: whole spatial points per block (stencil form), or the sum-factorised plan
  if (P->sf_on) {
    SumFacPlan& sp = P->sf;
    sp.d = hp.d;
    sp.n_t = hp.n_t;
    sp.pt = hp.p_t;
    sp.ps = hp.p_s;
    for (int l = 0; l < hp.d; ++l) sp.n[l] = hp.n_s[l];
    sp.N = hp.N;
    sp.tband = P->TbL;
    sp.work_stride = P->n2 * P->max_nrhs;
    if (sumfac_plan_shape(sp, P->max_lds) != 0) {
      stfd_destroy(P);
      return STFD_EINVAL;
    }
    for (int l = 0; l < hp.d; ++l)
      if ((rc = upload(P, &sp.bands[l], sf_bands[l].data(), sf_bands[l].size()))) {
        stfd_destroy(P);
        return rc;
      }
    if ((rc = dev_alloc(P, &sp.work, size_t(hp.d == 3 ? 6 : 3) * size_t(sp.work_stride)))) {
      stfd_destroy(P);
      return rc;
    }
    P->mv_blocks = sp.last_grid;
  } else {
    P->mv_points = matvec_points_per_block(hp, P->n_cus);
    P->mv_blocks = (hp.N_s + P->mv_points - 1) / P->mv_points;
    if (P->mv_long) P->mv_blocks = (hp.N + kMvLongBlock - 1) / kMvLongBlock;
  }
  // row groups of every product from the heuristic (the autotune below may change them); the dot
  // partials are sized for one row group, the largest block count
  for (int prec = MP_F64; prec <= MP_BF16; ++prec)
    for (int l = 0; l < hp.d; ++l) {
      const int rt = mode_product_row_groups(hp.n_s[l], mp_inner(hp, l), mp_outer(hp, l));
      // large launches take the wide form where the operand is one matrix (measured at 3D p = 3
      // 48^4: FP64 apply 532 -> 468 us, FP32 369 -> 305 us, BF16 321 -> 276 us)
      P->mp_rt[prec][l] = (rt == 2 && !(l == 0 && P->u_slice0)) ? kMpWide : rt;
    }
  set_last_blocks(P);
  P->max_parts = std::max<int64_t>(std::max<int64_t>(P->mv_blocks, mp_last_blocks_bound(P)), kVecGrid);
  if ((rc = dev_alloc(P, &P->parts, size_t(6) * P->max_parts * P->max_nrhs)) ||
      (rc = dev_alloc(P, &P->sc, size_t(P->max_nrhs))) || (rc = dev_alloc(P, &P->done, size_t(P->max_nrhs))) ||
      (rc = dev_alloc(P, &P->ctr, size_t(1)))) {
    stfd_destroy(P);
    return rc;
  }
  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&P->sc_host), sizeof(PcgScalars) * kLag * P->max_nrhs);
  if (e != hipSuccess) {
    g_last_hip_error = int(e);
    P->sc_host = nullptr;
    stfd_destroy(P);
    return STFD_ENOMEM;
  }
  e = hipHostGetDevicePointer(reinterpret_cast<void**>(&P->sc_host_dev), P->sc_host, 0);
  if (e != hipSuccess) {
    g_last_hip_error = int(e);
    stfd_destroy(P);
    return STFD_EHIP;
  }
  if (int he = load_plan_build(hp, P->load)) {
    stfd_destroy(P);
    if (he == -2) return STFD_ENOTSPD;
    g_last_hip_error = he;
    return STFD_EHIP;
  }
  stfd::set_plan_model(P);
  e = hipHostMalloc(reinterpret_cast<void**>(&P->lift_status_host), sizeof(int));
  if (e != hipSuccess) {
    g_last_hip_error = int(e);
    P->lift_status_host = nullptr;
    stfd_destroy(P);
    return STFD_ENOMEM;
  }
  e = hipHostGetDevicePointer(reinterpret_cast<void**>(&P->lift_status_dev), P->lift_status_host, 0);
  if (e != hipSuccess) {
    g_last_hip_error = int(e);
    stfd_destroy(P);
    return STFD_EHIP;
  }
  // device address of the allocation-free apply's scratch on this device
  {
    void* sp = nullptr;
    if ((rc = scratch_address(&sp))) {
      stfd_destroy(P);
      return rc;
    }
  }
  // right-hand side workspace: the Gauss-grid scratch of one right-hand side and the lifting
  // tensors of max_nrhs (stfd_load_vector allocates nothing)
  if (!desc->no_rhs_workspace) {
    if ((rc = dev_alloc(P, &P->rhs_work, rhs_work_reals(P->load))) ||
        (rc = dev_alloc(P, &P->rhs_lift, size_t(2) * size_t(P->load.n_full) * size_t(P->max_nrhs)))) {
      stfd_destroy(P);
      return rc;
    }
  }
  if (desc->autotune) {
    const auto t0 = std::chrono::steady_clock::now();
    TuneClock C;
    if ((rc = C.init())) {
      stfd_destroy(P);
      return rc;
    }
    STFD_HIP(hipMemsetAsync(P->vec[0], 0, sizeof(double) * size_t(P->n2), C.s));
    if ((rc = tune_mode_products(P, C, P->vec[0], P->vec[1])) ||
        (rc = setup_fused(P, desc->fused_segment_length, true, &C, P->vec[0], P->vec[1]))) {
      stfd_destroy(P);
      return rc;
    }
    STFD_HIP(hipStreamSynchronize(C.s));
    P->tune_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    P->autotuned = true;
  } else if ((rc = setup_fused(P, desc->fused_segment_length, false, nullptr, nullptr, nullptr))) {
    stfd_destroy(P);
    return rc;
  }
  *out = P;
  return STFD_OK;
}

int stfd_set_lift_max_iterations(stfd_problem* P, int max_iter) {
  if (!P || max_iter < 1) return STFD_EINVAL;
  P->lift_max_iter = max_iter;
  return STFD_OK;
}

int stfd_load_vector(const stfd_problem* P, const void* f_q_dev, const void* u0_q_dev,
                     const void* const* dirichlet_q_dev, void* fbar_dev, double* lift, int64_t nrhs, void* stream) {
  if (!P || !fbar_dev || nrhs < 1 || nrhs > P->max_nrhs || !P->rhs_work) return STFD_EINVAL;
  const HostProblem& hp = P->hp;
  const LoadPlan& plan = P->load;
  hipStream_t s = static_cast<hipStream_t>(stream);
  size_t grid = 1, nq_s = 1;
  for (int a = 0; a < plan.na; ++a) grid *= size_t(plan.Q[a]);
  for (int a = 1; a < plan.na; ++a) nq_s *= size_t(plan.Q[a]);
  // face grids: time fastest, then the tangent spatial directions
  size_t nq_face[6];
  for (int l = 0; l < hp.d; ++l) {
    size_t c = size_t(plan.Q[0]);
    for (int k = 0; k < hp.d; ++k)
      if (k != l) c *= size_t(plan.Q[k + 1]);
    nq_face[2 * l] = nq_face[2 * l + 1] = c;
  }
  const size_t nfull = size_t(plan.n_full);
  int rc = STFD_OK;
  const double* faces[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  if (hp.time_final) {
    // ultraweak method: (f, B_I) + i (u_0, B_I(0)), homogeneous Dirichlet data, no lifting
    if (dirichlet_q_dev)
      for (int k = 0; k < 2 * hp.d; ++k)
        if (dirichlet_q_dev[k]) return STFD_EINVAL;
    for (int64_t r = 0; r < nrhs; ++r) {
      const double* u0 = u0_q_dev ? static_cast<const double*>(u0_q_dev) + size_t(r) * 2 * nq_s : nullptr;
      const double* fq = f_q_dev ? static_cast<const double*>(f_q_dev) + size_t(r) * 2 * grid : nullptr;
      double* out = static_cast<double*>(fbar_dev) + size_t(r) * P->n2;
      const int he = ultraweak_rhs_device(hp, plan, fq, u0, out, P->rhs_work, s);
      if (he != 0) {
        g_last_hip_error = he;
        return STFD_EHIP;
      }
    }
    const hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      g_last_hip_error = int(e);
      return STFD_EHIP;
    }
    if (lift) std::memset(lift, 0, nfull * 2 * sizeof(double) * size_t(nrhs));
    return STFD_OK;
  }
  for (int64_t r = 0; r < nrhs && (rc == STFD_OK || rc == STFD_NOT_CONVERGED); ++r) {
    for (int k = 0; k < 2 * hp.d; ++k)
      faces[k] = (dirichlet_q_dev && dirichlet_q_dev[k])
                     ? static_cast<const double*>(dirichlet_q_dev[k]) + size_t(r) * 2 * nq_face[k]
                     : nullptr;
    const double* u0 = u0_q_dev ? static_cast<const double*>(u0_q_dev) + size_t(r) * 2 * nq_s : nullptr;
    const double* fq = f_q_dev ? static_cast<const double*>(f_q_dev) + size_t(r) * 2 * grid : nullptr;
    double* out = static_cast<double*>(fbar_dev) + size_t(r) * P->n2;
    double* G = P->rhs_lift + size_t(r) * 2 * nfull;
    *P->lift_status_host = 0;
    int he = rhs_device(hp, plan, fq, u0, faces, G, out, P->rhs_work, P->lift_status_dev, P->lift_status_host,
                        P->lift_max_iter, s);
    if (he == 0) he = int(hipStreamSynchronize(s));
    if (he != 0) {
      g_last_hip_error = he;
      rc = STFD_EHIP;
    } else if (*P->lift_status_host == 2) {
      rc = STFD_ENOTSPD;
    } else if (*P->lift_status_host == 3) {
      rc = STFD_NOT_CONVERGED;  // this right-hand side is assembled from the last lifting iterate
    }
  }
  if ((rc == STFD_OK || rc == STFD_NOT_CONVERGED) && lift) {
    hipError_t e = hipMemcpyAsync(lift, P->rhs_lift, nfull * 2 * sizeof(double) * size_t(nrhs),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      g_last_hip_error = int(e);
      rc = STFD_EHIP;
    }
  }
  return rc;
}

int stfd_sizes(const stfd_problem* P, int64_t* n_t, int64_t n_s[3], int64_t* n_dof) {
  if (!P) return STFD_EINVAL;
  if (n_t) *n_t = P->hp.n_t;
  if (n_s)
    for (int l = 0; l < 3; ++l) n_s[l] = (l < P->hp.d) ? P->hp.n_s[l] : 1;
  if (n_dof) *n_dof = P->hp.N;
  return STFD_OK;
}

int stfd_get_tuning(const stfd_problem* P, stfd_tuning* out) {
  if (!P || !out) return STFD_EINVAL;
  std::memset(out, 0, sizeof(*out));
  out->autotuned = P->autotuned ? 1 : 0;
  for (int prec = 0; prec < 3; ++prec)
    for (int l = 0; l < 3; ++l) out->mode_product_row_groups[prec][l] = l < P->hp.d ? P->mp_rt[prec][l] : 0;
  out->time_segment_length = P->ts_len;
  out->time_transfers_in_kernel = P->ts_mode >= 1 ? 1 : 0;
  out->time_factors_in_kernel = P->ts_mode == 2 ? 1 : 0;
  out->tune_ms = P->tune_ms;
  out->fused_time = P->fz_on ? 1 : 0;
  out->fused_segment_length = P->fz_len;
  out->fused_factors_in_kernel = P->fz_len && P->fz_mode == 2 ? 1 : 0;
  return STFD_OK;
}

int stfd_set_tuning(stfd_problem* P, const stfd_tuning* in) {
  if (!P || !in) return STFD_EINVAL;
  const HostProblem& hp = P->hp;
  if (in->time_segment_length != P->ts_len || in->time_transfers_in_kernel != (P->ts_mode >= 1 ? 1 : 0) ||
      in->time_factors_in_kernel != (P->ts_mode == 2 ? 1 : 0))
    return STFD_EINVAL;
  if (in->fused_segment_length != P->fz_len ||
      in->fused_factors_in_kernel != (P->fz_len && P->fz_mode == 2 ? 1 : 0) ||
      (in->fused_time != 0 && in->fused_time != 1) || (in->fused_time && !P->fz_len))
    return STFD_EINVAL;
  for (int prec = 0; prec < 3; ++prec)
    for (int l = 0; l < hp.d; ++l) {
      const int rt = in->mode_product_row_groups[prec][l];
      if (rt < 1 || rt > kMpWide || (rt >= 2 && hp.n_s[l] > 80) || (rt == kMpWide && l == 0 && P->u_slice0))
        return STFD_EINVAL;
    }
  for (int prec = 0; prec < 3; ++prec)
    for (int l = 0; l < hp.d; ++l) P->mp_rt[prec][l] = in->mode_product_row_groups[prec][l];
  P->fz_on = in->fused_time != 0;
  set_last_blocks(P);
  graph_cache_clear(P);  // captured iterations hold the previous launch shapes
  return STFD_OK;
}

int stfd_get_precond_shift(const stfd_problem* P, double* c) {
  if (!P || !c) return STFD_EINVAL;
  *c = P->hp.shift;
  return STFD_OK;
}

int stfd_get_pencil(const stfd_problem* P, int l, double* U, double* lambda) {
  if (!P || l < 0 || l >= P->hp.d) return STFD_EINVAL;
  if (U) std::memcpy(U, P->hp.U[l].data(), P->hp.U[l].size() * sizeof(double));
  if (lambda) std::memcpy(lambda, P->hp.lam1[l].data(), P->hp.lam1[l].size() * sizeof(double));
  return STFD_OK;
}

int stfd_timing_begin(stfd_problem* P, int capacity) {
  if (!P || capacity < 1 || P->timing) return STFD_EINVAL;
  stfd::graph_cache_clear(P);  // captured iterations carry no timing events
  P->tev.assign(size_t(2) * capacity, nullptr);
  for (hipEvent_t& e : P->tev) {
    const hipError_t he = hipEventCreate(&e);
    if (he != hipSuccess) {
      for (hipEvent_t f : P->tev)
        if (f) (void)hipEventDestroy(f);
      P->tev.clear();
      g_last_hip_error = int(he);
      return STFD_EHIP;
    }
  }
  P->tev_used = 0;
  P->timing = true;
  return STFD_OK;
}

int stfd_timing_end(stfd_problem* P, double* total_ms, int64_t* launches) {
  if (!P || !P->timing) return STFD_EINVAL;
  stfd::graph_cache_clear(P);  // iterations captured while timing record its events
  double tot = 0.0;
  int rc = STFD_OK;
  for (size_t k = 0; k + 1 < P->tev_used; k += 2) {
    float ms = 0.0f;
    hipError_t he = hipEventSynchronize(P->tev[k + 1]);
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, P->tev[k], P->tev[k + 1]);
    if (he != hipSuccess) {
      g_last_hip_error = int(he);
      rc = STFD_EHIP;
      break;
    }
    tot += ms;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = int64_t(P->tev_used / 2);
  for (hipEvent_t e : P->tev) (void)hipEventDestroy(e);
  P->tev.clear();
  P->tev_used = 0;
  P->timing = false;
  return rc;
}

int stfd_time_mode_product(stfd_problem* P, int direction, int precision, int reps, void* stream, double* avg_ms) {
  if (!P || !avg_ms || reps < 1 || direction < 0 || direction >= P->hp.d || precision < STFD_FP64 ||
      precision > STFD_BF16)
    return STFD_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const HostProblem& hp = P->hp;
  const int l = direction, n = hp.n_s[l];
  const int64_t inner = mp_inner(hp, l), outer = mp_outer(hp, l);
  const int64_t slice = l == 0 ? P->upk_slice[precision] : 0;
  // the forward product of one right-hand side in the applies' shape, from one work buffer into the
  // other (FP64: FP64 in and out, as the first product of an FP64 apply; otherwise FP32 in and out)
  auto launch = [&]() -> int {
    const int rt = P->mp_rt[precision][l];
    if (precision == STFD_FP64)
      return launch_mode_product<MP_F64, double, double>(P->work64[0], P->work64[1], P->Upk_fwd[MP_F64][l], n, inner,
                                                         outer, outer, nullptr, s, DotEpilogue(), slice, rt);
    if (precision == STFD_FP32)
      return launch_mode_product<MP_F32, float, float>(P->work32[0], P->work32[1], P->Upk_fwd[MP_F32][l], n, inner,
                                                       outer, outer, nullptr, s, DotEpilogue(), slice, rt);
    return launch_mode_product<MP_BF16, float, float>(P->work32[0], P->work32[1], P->Upk_fwd[MP_BF16][l], n, inner,
                                                      outer, outer, nullptr, s, DotEpilogue(), slice, rt);
  };
  int rc;
  for (int w = 0; w < 2; ++w)
    if ((rc = launch())) return rc;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) e = hipEventRecord(a, s);
  rc = STFD_OK;
  for (int k = 0; k < reps && e == hipSuccess && rc == STFD_OK; ++k) rc = launch();
  if (e == hipSuccess && rc == STFD_OK) e = hipEventRecord(b, s);
  if (e == hipSuccess && rc == STFD_OK) e = hipEventSynchronize(b);
  float ms = 0.0f;
  if (e == hipSuccess && rc == STFD_OK) e = hipEventElapsedTime(&ms, a, b);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (rc) return rc;
  if (e != hipSuccess) {
    g_last_hip_error = int(e);
    return STFD_EHIP;
  }
  *avg_ms = double(ms) / reps;
  return STFD_OK;
}

int stfd_apply_preconditioner(const stfd_problem* Pc, const void* r_dev, void* s_dev, int64_t nrhs, int precision,
                              void* stream) {
  stfd_problem* P = const_cast<stfd_problem*>(Pc);
  if (!P || !r_dev || !s_dev || nrhs < 1 || nrhs > P->max_nrhs) return STFD_EINVAL;
  if (precision < STFD_FP64 || precision > STFD_BF16) return STFD_EINVAL;
  return apply_dispatch(P, static_cast<const double*>(r_dev), static_cast<double*>(s_dev), nrhs, precision, nullptr,
                        static_cast<hipStream_t>(stream));
}

int stfd_apply_preconditioner_static(const stfd_problem* Pc, const void* r_dev, void* s_dev, int64_t nrhs,
                                     int precision, void* stream) {
  stfd_problem* P = const_cast<stfd_problem*>(Pc);
  if (!P || !r_dev || !s_dev || nrhs < 1) return STFD_EINVAL;
  if (precision < STFD_FP64 || precision > STFD_BF16) return STFD_EINVAL;
  // each intermediate holds 2 N nrhs reals of the working precision in one half of the scratch
  const size_t elem = apply_elem_bytes(precision);
  const size_t half = kScratchBytes / 2;
  if (uint64_t(nrhs) > uint64_t(half / (size_t(P->n2) * elem))) return STFD_EINVAL;
  void* base = nullptr;
  if (int rc = scratch_address(&base)) return rc;
  return apply_with_buffers(P, static_cast<const double*>(r_dev), static_cast<double*>(s_dev), nrhs, precision,
                            nullptr, static_cast<hipStream_t>(stream), base, static_cast<char*>(base) + half);
}

int stfd_matvec(const stfd_problem* Pc, const void* x_dev, void* y_dev, int64_t nrhs, void* stream) {
  stfd_problem* P = const_cast<stfd_problem*>(Pc);
  if (!P || !x_dev || !y_dev || nrhs < 1 || nrhs > P->max_nrhs || x_dev == y_dev) return STFD_EINVAL;
  return matvec_dispatch(P, static_cast<const double*>(x_dev), static_cast<double*>(y_dev), nrhs, nullptr, nullptr,
                         static_cast<hipStream_t>(stream));
}

namespace stfd {

// One solve of a batch: a problem handle with its own right-hand sides and work buffers.
struct PcgJob {
  stfd_problem* P;
  const double* f;
  double* x;
  int64_t nrhs;
};

// r_0 = f - A x_0, ||f||, z_0 = P^{-1} r_0, p_0 = z_0, <r_0, z_0>.
static int pcg_init(const PcgJob& J, int flags, int precision, double rtol, hipStream_t s) {
  stfd_problem* P = J.P;
  double* r = P->vec[0];
  double* z = P->vec[1];
  double* p = P->vec[3];
  double* q = P->vec[4];
  const int64_t n2 = P->n2;
  double* pa = P->parts;
  double* pb = pa + P->max_parts * P->max_nrhs;
  const dim3 vgrid(kVecGrid, unsigned(J.nrhs)), vblock(kVecBlock);
  int rc;
  if (flags & STFD_X0_GIVEN) {
    if ((rc = matvec_dispatch(P, J.x, q, J.nrhs, nullptr, nullptr, s))) return rc;
    int mode = 1;
    if (flags & STFD_X0_SCALED) {
      double* pc = pb + P->max_parts * P->max_nrhs;
      double* pd = pc + P->max_parts * P->max_nrhs;
      hipLaunchKernelGGL(dot_x0_kernel, vgrid, vblock, 0, s, J.x, J.f, q, n2, pb, pc, pd);
      hipLaunchKernelGGL(pcg_x0_scale_kernel, vgrid, vblock, 0, s, J.f, q, r, J.x, n2, pb, pc, pd, kVecGrid, pa,
                         P->sc);
      mode = 2;
    } else {
      hipLaunchKernelGGL(pcg_init_kernel, vgrid, vblock, 0, s, J.f, q, r, J.x, n2, pa);
    }
    hipLaunchKernelGGL(dot2_kernel, vgrid, vblock, 0, s, r, r, nullptr, n2, pb, nullptr, nullptr);
    hipLaunchKernelGGL(pcg_start_kernel, dim3(unsigned(J.nrhs)), vblock, 0, s, pa, pb, kVecGrid, P->sc, P->done, rtol,
                       P->ctr, mode);
    if (mode == 2) {
      hipLaunchKernelGGL(pcg_x0_revert_kernel, vgrid, vblock, 0, s, J.f, r, J.x, n2, (const PcgScalars*)P->sc);
      hipLaunchKernelGGL(pcg_x0_revert_finish_kernel, dim3(unsigned((J.nrhs + 63) / 64)), dim3(64), 0, s, P->sc,
                         P->done, int(J.nrhs), rtol);
    }
  } else {
    hipLaunchKernelGGL(pcg_init_kernel, vgrid, vblock, 0, s, J.f, nullptr, r, J.x, n2, pa);
    hipLaunchKernelGGL(pcg_start_kernel, dim3(unsigned(J.nrhs)), vblock, 0, s, pa, nullptr, kVecGrid, P->sc, P->done,
                       rtol, P->ctr, 0);
  }
  STFD_HIP(hipGetLastError());
  if ((rc = apply_dispatch(P, r, z, J.nrhs, precision, P->done, s))) return rc;
  hipLaunchKernelGGL(dot2_kernel, vgrid, vblock, 0, s, r, z, nullptr, n2, pa, nullptr, P->done);
  hipLaunchKernelGGL(pcg_first_p_kernel, vgrid, vblock, 0, s, z, p, n2, pa, kVecGrid, P->sc, P->done);
  STFD_HIP(hipGetLastError());
  return STFD_OK;
}

// Iteration k (parity = k & 1): q = A p (+<p,q>), x/r update (+||r||^2),
// z_new = P^{-1} r (+<r,z_new>, <r,z_old>), end-of-iteration test and p update.  The
// iteration index, the ring slot and every scalar live on the device, so the same launch
// sequence serves every iteration of a parity (and can be captured into a graph).
static int pcg_iteration(const PcgJob& J, int parity, int precision, int maxit, double rtol, hipStream_t s) {
  stfd_problem* P = J.P;
  double* r = P->vec[0];
  double* zold = P->vec[1 + parity];
  double* znew = P->vec[2 - parity];
  double* p = P->vec[3];
  double* q = P->vec[4];
  const int64_t n2 = P->n2;
  const int64_t mp = P->max_parts;
  double* pa = P->parts;               // <r, z_new> partials (last mode product)
  double* pb = pa + mp * P->max_nrhs;  // <r, z_old> partials
  double* pc = pb + mp * P->max_nrhs;  // ||r||^2 partials (pcg_update_xr)
  double* pd = pc + mp * P->max_nrhs;  // <p, A p> partials (matvec)
  const dim3 vgrid(kVecGrid, unsigned(J.nrhs)), vblock(kVecBlock);
  // With one right-hand side the matvec and apply kernels skip the done-flag test: the few
  // iterations launched after convergence only overwrite q and z_new, while x, r and p are
  // guarded by the flag in pcg_update_xr / pcg_end_iter.
  const int* dflag = J.nrhs > 1 ? P->done : nullptr;
  int rc;
  if ((rc = matvec_dispatch(P, p, q, J.nrhs, pd, dflag, s))) return rc;
  hipLaunchKernelGGL(pcg_update_xr_kernel, vgrid, vblock, 0, s, p, q, J.x, r, n2, pd, int(P->mv_blocks), P->sc,
                     parity, pc, P->done, P->ctr);
  DotEpilogue ep;
  ep.r = r;
  ep.zold = zold;
  ep.part_a = pa;
  ep.part_b = pb;
  if ((rc = apply_dispatch(P, r, znew, J.nrhs, precision, dflag, s, ep))) return rc;
  // blocks of the end-of-iteration kernel: one per kEndBlock elements, at most kEndGrid (every block
  // repeats the reduction, so small systems take few)
  const unsigned egrid = unsigned(std::min<int64_t>(kEndGrid, std::max<int64_t>(1, (n2 / 2 + kEndBlock - 1) / kEndBlock)));
  hipLaunchKernelGGL(pcg_end_iter_kernel, dim3(egrid, unsigned(J.nrhs)), dim3(kEndBlock), 0, s, znew, p, n2, pc,
                     kVecGrid, pa, pb, int(P->mp_last_blocks[precision]), P->sc, parity, P->done, maxit, rtol, P->sc_host_dev,
                     P->max_nrhs, (const int*)P->ctr);
  STFD_HIP(hipGetLastError());
  return STFD_OK;
}

// true residual ||f - A x|| / ||f|| and the per-system results
static int pcg_finish(const PcgJob& J, stfd_pcg_info* info, hipStream_t s) {
  stfd_problem* P = J.P;
  double* q = P->vec[4];
  double* pa = P->parts;
  const dim3 vgrid(kVecGrid, unsigned(J.nrhs)), vblock(kVecBlock);
  int rc;
  if ((rc = matvec_dispatch(P, J.x, q, J.nrhs, nullptr, nullptr, s))) return rc;
  hipLaunchKernelGGL(resid_norm_kernel, vgrid, vblock, 0, s, J.f, q, P->n2, pa);
  hipLaunchKernelGGL(pcg_finish_kernel, dim3(unsigned(J.nrhs)), vblock, 0, s, pa, kVecGrid, P->sc);
  STFD_HIP(hipGetLastError());
  std::vector<PcgScalars> fin(J.nrhs);
  STFD_HIP(hipMemcpyAsync(fin.data(), P->sc, sizeof(PcgScalars) * J.nrhs, hipMemcpyDeviceToHost, s));
  STFD_HIP(hipStreamSynchronize(s));
  int status = STFD_OK;
  for (int64_t rr = 0; rr < J.nrhs; ++rr) {
    const PcgScalars& sc = fin[rr];
    int st = sc.status;
    if (!sc.done && st == STFD_OK) st = STFD_NOT_CONVERGED;  // maxit == 0 with a non-converged start
    if (info) {
      info[rr].iters = sc.iters;
      info[rr].status = st;
      info[rr].rel_res = sc.res;
      info[rr].true_rel_res = sc.true_res;
      info[rr].x0_scale = sc.x0_scale;
    }
    if (st == STFD_EBREAKDOWN) status = STFD_EBREAKDOWN;
    else if (st == STFD_NOT_CONVERGED && status == STFD_OK) status = STFD_NOT_CONVERGED;
  }
  return status;
}

// Captured iteration graphs (one per parity) of a batch of solves: every job runs on its own
// stream forked from `s`, so the independent systems overlap on the device.
// The graphs are recorded on a private capture stream (the caller's stream may be the null
// stream, which cannot capture) and launched on the caller's stream.
struct IterationGraphs {
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  hipStream_t cap = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  ~IterationGraphs() {
    for (auto& e : exec)
      if (e) (void)hipGraphExecDestroy(e);
    if (cap) (void)hipStreamDestroy(cap);
    for (auto st : streams)
      if (st) (void)hipStreamDestroy(st);
    for (auto ev : events)
      if (ev) (void)hipEventDestroy(ev);
  }
};

static int capture_iterations(const std::vector<PcgJob>& jobs, int precision, int maxit, double rtol,
                              IterationGraphs& G) {
  const size_t nj = jobs.size();
  STFD_HIP(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
  hipStream_t s = G.cap;
  if (nj > 1) {
    G.streams.resize(nj, nullptr);
    G.events.resize(nj + 1, nullptr);
    for (size_t k = 0; k < nj; ++k) STFD_HIP(hipStreamCreateWithFlags(&G.streams[k], hipStreamNonBlocking));
    for (size_t k = 0; k <= nj; ++k) STFD_HIP(hipEventCreateWithFlags(&G.events[k], hipEventDisableTiming));
  }
  for (int par = 0; par < 2; ++par) {
    hipGraph_t graph = nullptr;
    STFD_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = STFD_OK;
    if (nj == 1) {
      rc = pcg_iteration(jobs[0], par, precision, maxit, rtol, s);
    } else {
      hipError_t e = hipEventRecord(G.events[nj], s);
      for (size_t k = 0; k < nj && rc == STFD_OK && e == hipSuccess; ++k) {
        e = hipStreamWaitEvent(G.streams[k], G.events[nj], 0);
        if (e == hipSuccess) rc = pcg_iteration(jobs[k], par, precision, maxit, rtol, G.streams[k]);
        if (rc == STFD_OK && e == hipSuccess) e = hipEventRecord(G.events[k], G.streams[k]);
        if (rc == STFD_OK && e == hipSuccess) e = hipStreamWaitEvent(s, G.events[k], 0);
      }
      if (e != hipSuccess && rc == STFD_OK) {
        g_last_hip_error = int(e);
        rc = STFD_EHIP;
      }
    }
    hipError_t ec = hipStreamEndCapture(s, &graph);
    if (rc != STFD_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (ec != hipSuccess) {
      g_last_hip_error = int(ec);
      return STFD_EHIP;
    }
    hipError_t ei = hipGraphInstantiateWithFlags(&G.exec[par], graph, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      g_last_hip_error = int(ei);
      return STFD_EHIP;
    }
  }
  return STFD_OK;
}

// Captured iterations of one job, from the handle's cache or captured now and cached (at most
// kGraphCache per handle; the least recently used is dropped).  The graphs hold the job's buffers,
// sizes, precision and stopping parameters; anything else they depend on (launch shapes, potential,
// timing) drops the whole cache when it changes (graph_cache_clear).  *out points into the cache:
// valid until the next lookup or clear on this handle (one lookup per handle and solve).
constexpr size_t kGraphCache = 4;
static void graph_cache_clear(stfd_problem* P) {
  for (auto& g : P->graphs)
    for (auto& e : g.exec)
      if (e) (void)hipGraphExecDestroy(e);
  P->graphs.clear();
}
static int cached_iterations(const PcgJob& J, int precision, int maxit, double rtol, hipGraphExec_t** out) {
  stfd_problem* P = J.P;
  for (auto& g : P->graphs)
    if (g.f == J.f && g.x == J.x && g.nrhs == J.nrhs && g.precision == precision && g.maxit == maxit &&
        g.rtol == rtol) {
      g.used = ++P->graph_clock;
      *out = g.exec;
      return STFD_OK;
    }
  IterationGraphs G;
  const std::vector<PcgJob> one(1, J);
  if (int rc = capture_iterations(one, precision, maxit, rtol, G)) return rc;
  if (P->graphs.size() >= kGraphCache) {
    auto lru = std::min_element(P->graphs.begin(), P->graphs.end(),
                                [](const auto& a, const auto& b) { return a.used < b.used; });
    for (auto& e : lru->exec)
      if (e) (void)hipGraphExecDestroy(e);
    P->graphs.erase(lru);
  }
  stfd_problem::CachedIterations c;
  c.f = J.f;
  c.x = J.x;
  c.nrhs = J.nrhs;
  c.precision = precision;
  c.maxit = maxit;
  c.rtol = rtol;
  for (int k = 0; k < 2; ++k) {
    c.exec[k] = G.exec[k];
    G.exec[k] = nullptr;  // owned by the cache now
  }
  c.used = ++P->graph_clock;
  P->graphs.push_back(c);
  *out = P->graphs.back().exec;
  return STFD_OK;
}

// Shared driver of stfd_pcg_solve and stfd_pcg_solve_batched.  The host launches iteration k
// (directly or as a graph), records an event, and before iteration k reads the pinned ring
// slot that iteration k - kLag wrote; the loop ends when every system of every job is done.
static int pcg_run(std::vector<PcgJob>& jobs, double rtol, int maxit, int flags, int precision, bool use_graph,
                   stfd_pcg_info* info, hipStream_t s) {
  int rc;
  for (const PcgJob& J : jobs)
    if ((rc = pcg_init(J, flags, precision, rtol, s))) return rc;
  IterationGraphs G;
  hipGraphExec_t* exec = G.exec;
  if (use_graph && maxit > 0) {
    if (jobs.size() == 1) {
      if ((rc = cached_iterations(jobs[0], precision, maxit, rtol, &exec))) return rc;
    } else if ((rc = capture_iterations(jobs, precision, maxit, rtol, G))) {
      return rc;
    }
  }
  std::vector<hipEvent_t> ev(kLag, nullptr);
  auto cleanup = [&]() {
    for (auto e : ev)
      if (e) (void)hipEventDestroy(e);
  };
  for (int k = 0; k < kLag; ++k)
    if (hipEventCreateWithFlags(&ev[k], hipEventDisableTiming) != hipSuccess) {
      cleanup();
      return STFD_EHIP;
    }
  for (int k = 0; k < maxit; ++k) {
    if (k >= kLag) {
      const int slot = (k - kLag) % kLag;
      if (hipEventSynchronize(ev[slot]) != hipSuccess) {
        cleanup();
        return STFD_EHIP;
      }
      bool all = true;
      for (const PcgJob& J : jobs)
        for (int64_t rr = 0; rr < J.nrhs; ++rr) all = all && J.P->sc_host[slot * J.P->max_nrhs + rr].done;
      if (all) break;
    }
    const int par = k & 1;
    if (use_graph) {
      if (hipGraphLaunch(exec[par], s) != hipSuccess) {
        cleanup();
        return STFD_EHIP;
      }
    } else {
      for (const PcgJob& J : jobs)
        if ((rc = pcg_iteration(J, par, precision, maxit, rtol, s))) {
          cleanup();
          return rc;
        }
    }
    if (hipEventRecord(ev[k % kLag], s) != hipSuccess) {
      cleanup();
      return STFD_EHIP;
    }
  }
  cleanup();
  int status = STFD_OK;
  int64_t off = 0;
  for (const PcgJob& J : jobs) {
    const int st = pcg_finish(J, info ? info + off : nullptr, s);
    off += J.nrhs;
    if (st < 0) return st;
    if (st == STFD_NOT_CONVERGED && status == STFD_OK) status = st;
  }
  for (int64_t k = 0; k < off && info; ++k)
    if (info[k].status == STFD_EBREAKDOWN) return STFD_EBREAKDOWN;
  return status;
}

// Batched driver: every job runs on its handle's own stream, forked from and joined back into `s`,
// so that the grids execute concurrently (a multi-stream graph is replayed with its branches one
// after the other, which leaves the small latency-bound grids serialised behind the large one).
// Each job keeps kLag iterations in flight and stops at its own convergence: the host polls the
// jobs' events without blocking and launches the next iteration of whichever job may proceed.
// graph: each job's iteration is a captured linear graph launched on the job's stream.
static int pcg_run_streams(std::vector<PcgJob>& jobs, double rtol, int maxit, int flags, int precision, bool graph,
                           stfd_pcg_info* info, hipStream_t s) {
  const size_t nj = jobs.size();
  for (PcgJob& J : jobs) {
    stfd_problem* P = J.P;
    if (!P->job_stream) STFD_HIP(hipStreamCreateWithFlags(&P->job_stream, hipStreamNonBlocking));
    for (hipEvent_t& e : P->job_ev)
      if (!e) STFD_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  // fork: every job stream starts after the work already on s
  hipEvent_t fork = jobs[0].P->job_ev[kLag];
  STFD_HIP(hipEventRecord(fork, s));
  for (PcgJob& J : jobs) STFD_HIP(hipStreamWaitEvent(J.P->job_stream, fork, 0));
  int rc;
  for (PcgJob& J : jobs)
    if ((rc = pcg_init(J, flags, precision, rtol, J.P->job_stream))) return rc;
  std::vector<hipGraphExec_t*> G(graph && maxit > 0 ? nj : 0, nullptr);
  for (size_t j = 0; j < G.size(); ++j)
    if ((rc = cached_iterations(jobs[j], precision, maxit, rtol, &G[j]))) return rc;
  std::vector<int> launched(nj, 0);
  std::vector<char> active(nj, maxit > 0 ? 1 : 0);
  size_t n_active = maxit > 0 ? nj : 0;
  while (n_active > 0) {
    bool progressed = false;
    for (size_t j = 0; j < nj; ++j) {
      if (!active[j]) continue;
      PcgJob& J = jobs[j];
      stfd_problem* P = J.P;
      const int k = launched[j];
      bool stop = k >= maxit;
      if (!stop && k >= kLag) {
        const int slot = (k - kLag) % kLag;
        const hipError_t q = hipEventQuery(P->job_ev[slot]);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) {
          g_last_hip_error = int(q);
          return STFD_EHIP;
        }
        bool all = true;
        for (int64_t rr = 0; rr < J.nrhs; ++rr) all = all && P->sc_host[slot * P->max_nrhs + rr].done;
        stop = all;
      }
      if (stop) {
        active[j] = 0;
        --n_active;
        continue;
      }
      if (graph) {
        STFD_HIP(hipGraphLaunch(G[j][k & 1], P->job_stream));
      } else if ((rc = pcg_iteration(J, k & 1, precision, maxit, rtol, P->job_stream))) {
        return rc;
      }
      STFD_HIP(hipEventRecord(P->job_ev[k % kLag], P->job_stream));
      launched[j] = k + 1;
      progressed = true;
    }
    if (!progressed && n_active > 0) std::this_thread::yield();
  }
  int status = STFD_OK;
  int64_t off = 0;
  for (PcgJob& J : jobs) {
    const int st = pcg_finish(J, info ? info + off : nullptr, J.P->job_stream);
    off += J.nrhs;
    if (st < 0) return st;
    if (st == STFD_NOT_CONVERGED && status == STFD_OK) status = st;
  }
  // join: later work on s sees the solutions
  for (PcgJob& J : jobs) {
    STFD_HIP(hipEventRecord(J.P->job_ev[kLag], J.P->job_stream));
    STFD_HIP(hipStreamWaitEvent(s, J.P->job_ev[kLag], 0));
  }
  for (int64_t k = 0; k < off && info; ++k)
    if (info[k].status == STFD_EBREAKDOWN) return STFD_EBREAKDOWN;
  return status;
}

}  // namespace stfd

int stfd_pcg_solve(const stfd_problem* Pc, const void* f_dev, void* u_dev, int64_t nrhs, double rtol, int maxit,
                   int flags, int precision, stfd_pcg_info* info, void* stream) {
  stfd_problem* P = const_cast<stfd_problem*>(Pc);
  if (!P || !f_dev || !u_dev || nrhs < 1 || nrhs > P->max_nrhs || maxit < 0 || !(rtol >= 0.0)) return STFD_EINVAL;
  const int x0 = flags & ~STFD_PCG_GRAPH;
  if (x0 != STFD_X0_ZERO && x0 != STFD_X0_GIVEN && x0 != (STFD_X0_GIVEN | STFD_X0_SCALED)) return STFD_EINVAL;
  if (precision < STFD_FP64 || precision > STFD_BF16) return STFD_EINVAL;
  std::vector<PcgJob> jobs(1);
  jobs[0].P = P;
  jobs[0].f = static_cast<const double*>(f_dev);
  jobs[0].x = static_cast<double*>(u_dev);
  jobs[0].nrhs = nrhs;
  std::vector<stfd_pcg_info> tmp(info ? 0 : size_t(nrhs));
  return pcg_run(jobs, rtol, maxit, x0, precision, (flags & STFD_PCG_GRAPH) != 0, info ? info : tmp.data(),
                 static_cast<hipStream_t>(stream));
}

int stfd_pcg_solve_batched(const stfd_problem* const* probs, int count, const void* const* f_dev,
                           void* const* u_dev, const int64_t* nrhs, double rtol, int maxit, int flags,
                           int precision, stfd_pcg_info* info, void* stream) {
  if (!probs || !f_dev || !u_dev || !nrhs || count < 1 || count > 64 || maxit < 0 || !(rtol >= 0.0))
    return STFD_EINVAL;
  const int x0 = flags & ~STFD_PCG_GRAPH;
  if (x0 != STFD_X0_ZERO && x0 != STFD_X0_GIVEN && x0 != (STFD_X0_GIVEN | STFD_X0_SCALED)) return STFD_EINVAL;
  if (precision < STFD_FP64 || precision > STFD_BF16) return STFD_EINVAL;
  std::vector<PcgJob> jobs(static_cast<size_t>(count));
  int64_t total = 0;
  for (int k = 0; k < count; ++k) {
    stfd_problem* P = const_cast<stfd_problem*>(probs[k]);
    if (!P || !f_dev[k] || !u_dev[k] || nrhs[k] < 1 || nrhs[k] > P->max_nrhs) return STFD_EINVAL;
    for (int j = 0; j < k; ++j)
      if (jobs[size_t(j)].P == P) return STFD_EINVAL;  // one job per handle: it owns one set of work buffers
    jobs[size_t(k)].P = P;
    jobs[size_t(k)].f = static_cast<const double*>(f_dev[k]);
    jobs[size_t(k)].x = static_cast<double*>(u_dev[k]);
    jobs[size_t(k)].nrhs = nrhs[k];
    total += nrhs[k];
  }
  std::vector<stfd_pcg_info> tmp(info ? 0 : size_t(total));
  return pcg_run_streams(jobs, rtol, maxit, x0, precision, (flags & STFD_PCG_GRAPH) != 0, info ? info : tmp.data(),
                         static_cast<hipStream_t>(stream));
}

#ifdef STFD_PHASE_TIMING
int stfd_debug_phase_times(unsigned long long* out) {
  STFD_HIP(hipDeviceSynchronize());
  STFD_HIP(hipMemcpyFromSymbol(out, HIP_SYMBOL(g_phase), sizeof(g_phase)));
  STFD_HIP(hipMemcpyFromSymbol(out + 4096 * 8, HIP_SYMBOL(g_cycles), sizeof(g_cycles)));
  return STFD_OK;
}
#endif

int stfd_debug_mfma_layout(double* out64, float* out32, float* outbf) {
  if (!out64 || !out32 || !outbf) return STFD_EINVAL;
  double* d64 = nullptr;
  float* d32 = nullptr;
  float* dbf = nullptr;
  STFD_HIP(hipMalloc(&d64, 256 * sizeof(double)));
  STFD_HIP(hipMalloc(&d32, 256 * sizeof(float)));
  STFD_HIP(hipMalloc(&dbf, 256 * sizeof(float)));
  hipLaunchKernelGGL(mfma_layout_kernel, dim3(1), dim3(64), 0, 0, d64, d32, dbf);
  STFD_HIP(hipGetLastError());
  STFD_HIP(hipMemcpy(out64, d64, 256 * sizeof(double), hipMemcpyDeviceToHost));
  STFD_HIP(hipMemcpy(out32, d32, 256 * sizeof(float), hipMemcpyDeviceToHost));
  STFD_HIP(hipMemcpy(outbf, dbf, 256 * sizeof(float), hipMemcpyDeviceToHost));
  (void)hipFree(d64);
  (void)hipFree(d32);
  (void)hipFree(dbf);
  return STFD_OK;
}

}  // extern "C"
