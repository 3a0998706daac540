// Right-hand side of the least-squares system with lifting (Sections 2.2, 4.3).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "host_setup.h"

namespace stfd {

// One face of Gamma: the slice of full coefficients whose index along
// `normal_axis` equals `normal_index` (axis 0 = time, l + 1 = x_l).  Face-local
// entries are ordered with the tangent axes fastest first.
struct LiftFace {
  int normal_axis = 0, normal_index = 0;
  int n_tan = 0;
  int tan_axis[3] = {0, 0, 0};
  int dims[3] = {1, 1, 1};
  int64_t size = 0;    // product of dims
  int64_t offset = 0;  // into packed per-face buffers
};

struct LiftFaces {
  int count = 0;       // 1 + 2 d
  int na = 0;          // d + 1
  int m[4] = {1, 1, 1, 1};        // full basis size per axis
  int p[4] = {0, 0, 0, 0};        // degree per axis
  int64_t stride[4] = {0, 0, 0, 0};
  int64_t total = 0;   // sum of face sizes
  LiftFace f[7];
};

// Device data for the right-hand side, uploaded once per problem.
//   eval[a][r]: Q_a x m_a, [q][i] = b_i^(r)(x_q)                 (full basis)
//   load[a][r]: n_a x Q_a, [i][q] = w_q b_{i+1}^(r)(x_q)         (free basis)
//   wfull[a]:   m_a x Q_a, [i][q] = w_q b_i(x_q)                 (full basis, face data)
// with the non-zero column range of each row in *_lo / *_hi, and for the
// lifting: the fixed set (global indices), the global -> fixed position map,
// banded full 1D mass matrices [i][j - i + p] and their dense inverses.
struct LoadPlan {
  int na = 0;
  int Q[4] = {1, 1, 1, 1}, m[4] = {1, 1, 1, 1}, n[4] = {1, 1, 1, 1};
  double* eval[4][3] = {};
  int* eval_lo[4] = {};
  int* eval_hi[4] = {};
  double* load[4][3] = {};
  int* load_lo[4] = {};
  int* load_hi[4] = {};
  // time axis: bands of eval[0][r] and load[0][r] (r = 0, 1) transposed, band[u][row]
  double* tband_eval[2] = {};
  double* tband_load[2] = {};
  int tband_ew = 0, tband_lw = 0;
  double* wfull[4] = {};
  int* wfull_lo[4] = {};
  int* wfull_hi[4] = {};
  // spatial coefficients on the spatial Gauss grid (x_1 fastest), owned elsewhere:
  const double* Vq = nullptr;  // potential or nullptr
  const double* Jq = nullptr;  // Jacobian determinant or nullptr (1)
  int n_lap = 0;               // physical Laplacian = sum_k lap_c[k] D^{lap_ord[k]}
  int lap_ord[4][3] = {};
  const double* lap_c[4] = {};   // nullptr: 1
  const double* lap_cJ[4] = {};  // lap_c * J, nullptr: 1
  // lifting
  LiftFaces faces;
  int64_t n_fixed = 0, n_full = 0;
  int64_t* fixed = nullptr;   // [n_fixed] global index
  int* fixed_idx = nullptr;   // [n_fixed][4] its index along each axis (decoded once, on the host)
  int* pos = nullptr;         // [n_full] fixed position or -1
  double* Mband[4] = {};      // [m][2p + 1]
  double* Minv[4] = {};       // [m][m]
  int lift_blocks = 0;        // blocks of the fixed-set kernels
  std::vector<void*> allocs;
};

// Returns 0, -2 (a mass matrix is not positive definite), or a hipError_t (> 0).
int load_plan_build(const HostProblem& hp, LoadPlan& plan);
void load_plan_free(LoadPlan& plan);

// Device scratch (doubles) needed by rhs_device.
size_t rhs_work_reals(const LoadPlan& plan);

// Lifting and load vector of one right-hand side, all on `stream`:
//   u0_q (spatial grid) and faces[2l + side] (face grids) are device samples or nullptr,
//   f_q device samples on the space-time grid or nullptr,
//   G (out) the full coefficient tensor of the lifting, fbar (out) the free right-hand side.
// status_dev / status_host: device and host address of one pinned int that the lifting CG
// sets to 1 (converged), 2 (breakdown) or 3 (max_iter iterations without convergence); valid
// after a stream sync.  Returns 0 or a hipError_t.
int rhs_device(const HostProblem& hp, const LoadPlan& plan, const double* f_q, const double* u0_q,
               const double* const* faces, double* G, double* fbar, double* work, int* status_dev,
               volatile int* status_host, int max_iter, hipStream_t stream);

// Load vector of the ultraweak method (Section 4.4, eq. uw-discrete-system) for one right-hand
// side on the unit cube: fbar = (f, B_I) + i (u0, B_I(., 0)) over the free basis of W_h (time
// without its last function).  f_q / u0_q as for rhs_device (nullptr: zero).  Returns 0 or a
// hipError_t.
int ultraweak_rhs_device(const HostProblem& hp, const LoadPlan& plan, const double* f_q, const double* u0_q,
                         double* fbar, double* work, hipStream_t stream);

}  // namespace stfd
