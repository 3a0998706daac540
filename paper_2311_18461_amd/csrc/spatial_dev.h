// Device evaluation of the spatial factors from a SpatialModel (d <= 2), and the
// device copies of the model's coefficient arrays used by the load vector.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "spatial.h"

namespace stfd {

struct SpatialDevice {
  // per-direction basis tables of the spatial Gauss rule (d <= 2)
  double* B[2] = {nullptr, nullptr};  // [e][g][r][a]
  double* w[2] = {nullptr, nullptr};  // [e * q + g]
  int* first[2] = {nullptr, nullptr};
  int* elo[2] = {nullptr, nullptr};   // element range of each full function
  int* ehi[2] = {nullptr, nullptr};
  double* base = nullptr;             // V-free stencils [N_s][stencil][3] (unit cube) or nullptr
  std::vector<double*> arrays;        // device copies of SpatialModel::arrays
  std::vector<void*> allocs;          // tables and base (kept for the handle's lifetime)
};

// Upload the basis tables and the base stencils (interleaved [N_s][stencil][3]).  0 or hipError_t.
int spatial_device_init(const HostProblem& hp, const double* base_interleaved, SpatialDevice& sd);
// Upload the model's arrays (replacing earlier ones) and write Sc = base + terms on `stream`
// (d <= 2 on the device; d = 3 on the host, then uploaded).  0 or hipError_t.
int spatial_device_apply(const HostProblem& hp, const SpatialModel& m, SpatialDevice& sd, double* Sc_dev,
                         hipStream_t stream);
void spatial_device_free(SpatialDevice& sd);

}  // namespace stfd
