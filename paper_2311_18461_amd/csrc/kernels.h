// Device kernels of the space-time FD solver (CDNA4 / gfx950).
//
// Vector layout: complex values interleaved (re, im); a space-time tensor
// with time fastest, then x_1 .. x_d, then the right-hand side index
// (Section 3.3, vec operator).  Viewed as reals, a mode product along spatial
// direction l is a real GEMM: for every "outer" index o (directions above l
// and the right-hand side), Out[o][a][row] = sum_j In[o][j][row] U'[j][a],
// where `row` runs over the 2 n_t prod_{k<l} n_k contiguous reals below l.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace stfd {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef short s4_t __attribute__((ext_vector_type(4)));

constexpr int kMaxModeN = 128;   // largest n_l handled by the MFMA mode product
constexpr int kVecBlock = 256;   // threads of the BLAS-1 kernels
constexpr int kVecGrid = 1024;   // blocks per right-hand side of the BLAS-1 kernels

// Precision of a mode product: operands and accumulator.
enum { MP_F64 = 0, MP_F32 = 1, MP_BF16 = 2 };

struct ModeProductArgs {
  const void* in;
  void* out;
  const void* U;       // n x n operand, U'[j][a] = Uop[j*n + a]: FP64 for FP64 products, else FP32
  int64_t u_slice_stride;  // 0: one operand; else one per outer slice (o mod outer_per_rhs)
  int n;               // size of the contracted direction
  int64_t inner;       // contiguous reals below the direction
  int64_t outer;       // number of outer slices (directions above, times nrhs)
  int64_t outer_per_rhs;
  int64_t n_row_tiles;    // row tiles (16 RT rows, RT = 1 or 2) per outer slice, ceil(inner / (16 RT))
  int64_t tiles_per_rhs;  // outer_per_rhs * n_row_tiles
  int64_t tiles_pad;      // blocks per column group (row tiles, or groups of row tiles), padded to the XCD count
  int groups;             // 16-column groups computed by MFMA chains (mode_product_groups)
  const int* done;     // per right-hand side "converged" flags or nullptr
  // optional epilogue (FP64 output only): per-block partials of <r, out> and <r, zold>
  const double* dot_r;
  const double* dot_z;
  double* part_a;
  double* part_b;
};

}  // namespace stfd
