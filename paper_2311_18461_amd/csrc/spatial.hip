// Weighted forms of the spatial factors on the device (d <= 2).
//
// Entry (I, J) of  int w(xi) D^a phi_I D^b phi_J dxi  is a sum over the elements in the
// common support of phi_I and phi_J and their Gauss points.  One thread owns one stencil
// entry (row I, offset J - I) and sums every term of the model in a fixed order, so the
// result is deterministic and needs no atomics; the basis values come from per-direction
// tables [element][point][derivative][local function].
#include <hip/hip_runtime.h>

#include <algorithm>

#include "spatial_dev.h"

namespace stfd {

constexpr int kMaxWTerms = 40;

struct WTermDev {
  const double* cq;  // weight on the spatial grid (x_1 fastest) or nullptr (1)
  int a[2], b[2];
  double scale;
  int target;
};

struct WTermList {
  int count;
  WTermDev t[kMaxWTerms];
};

struct SpatialTables {
  const double* B[2];
  const double* w[2];
  const int* first[2];
  const int* elo[2];
  const int* ehi[2];
  int Q[2];
};

__global__ void __launch_bounds__(256) weighted_stencil_kernel(WTermList L, SpatialTables T, const double* base,
                                                               double* __restrict__ Sc, int d, int n1, int n2,
                                                               int64_t N_s, int stencil, int p, int q) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= N_s * stencil) return;
  const int64_t i = idx / stencil;
  const int s = int(idx - i * stencil);
  const int w2 = 2 * p + 1;
  const int il[2] = {int(i % n1), d > 1 ? int(i / n1) : 0};
  const int ol[2] = {s % w2 - p, d > 1 ? s / w2 - p : 0};
  const int nl[2] = {n1, n2};
  double acc[3] = {0.0, 0.0, 0.0};
  if (base)
    for (int k = 0; k < 3; ++k) acc[k] = base[idx * 3 + k];
  bool valid = true;
  int fi[2] = {0, 0}, fj[2] = {0, 0}, e0[2] = {0, 0}, e1[2] = {0, 0};
  for (int l = 0; l < 2; ++l) {
    if (l >= d) continue;
    const int j = il[l] + ol[l];
    if (j < 0 || j >= nl[l]) valid = false;
    fi[l] = il[l] + 1;  // full index (the first function is removed)
    fj[l] = min(max(j, 0), nl[l] - 1) + 1;
    e0[l] = max(T.elo[l][fi[l]], T.elo[l][fj[l]]);
    e1[l] = min(T.ehi[l][fi[l]], T.ehi[l][fj[l]]);
  }
  if (valid) {
    const int P1 = p + 1;
    for (int k = 0; k < L.count; ++k) {
      const WTermDev& t = L.t[k];
      double sum = 0.0;
      const int e2lo = d > 1 ? e0[1] : 0, e2hi = d > 1 ? e1[1] : 0;
      const int g2n = d > 1 ? q : 1;
      for (int e2 = e2lo; e2 <= e2hi; ++e2)
        for (int g2 = 0; g2 < g2n; ++g2) {
          double f2 = 1.0;
          int P2 = 0;
          if (d > 1) {
            const int a2 = fi[1] - T.first[1][e2], b2 = fj[1] - T.first[1][e2];
            const double* Bb = T.B[1] + (size_t(e2) * q + g2) * 3 * P1;
            f2 = T.w[1][e2 * q + g2] * Bb[t.a[1] * P1 + a2] * Bb[t.b[1] * P1 + b2];
            P2 = e2 * q + g2;
          }
          double inner = 0.0;
          for (int e1i = e0[0]; e1i <= e1[0]; ++e1i) {
            const int a1 = fi[0] - T.first[0][e1i], b1 = fj[0] - T.first[0][e1i];
            for (int g1 = 0; g1 < q; ++g1) {
              const double* Bb = T.B[0] + (size_t(e1i) * q + g1) * 3 * P1;
              const double f1 = T.w[0][e1i * q + g1] * Bb[t.a[0] * P1 + a1] * Bb[t.b[0] * P1 + b1];
              const double c = t.cq ? t.cq[int64_t(P2) * T.Q[0] + e1i * q + g1] : 1.0;
              inner = fma(f1, c, inner);
            }
          }
          sum = fma(f2, inner, sum);
        }
      acc[t.target] = fma(t.scale, sum, acc[t.target]);
    }
  }
  for (int k = 0; k < 3; ++k) Sc[idx * 3 + k] = acc[k];
}

namespace {

template <typename T>
int dev_upload(std::vector<void*>& owner, T** dst, const T* src, size_t n) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T));
  if (e != hipSuccess) return int(e);
  owner.push_back(p);
  e = hipMemcpy(p, src, n * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return int(e);
  *dst = static_cast<T*>(p);
  return 0;
}

}  // namespace

int spatial_device_init(const HostProblem& hp, const double* base_interleaved, SpatialDevice& sd) {
  for (int l = 0; l < std::min(hp.d, 2); ++l) {
    const Direction& D = hp.dir_s[l];
    std::vector<int> elo(size_t(D.m), D.n_el), ehi(size_t(D.m), -1);
    for (int e = 0; e < D.n_el; ++e)
      for (int a = 0; a <= D.p; ++a) {
        const int f = D.first[e] + a;
        elo[size_t(f)] = std::min(elo[size_t(f)], e);
        ehi[size_t(f)] = std::max(ehi[size_t(f)], e);
      }
    int rc;
    if ((rc = dev_upload(sd.allocs, &sd.B[l], D.basis.data(), D.basis.size())) ||
        (rc = dev_upload(sd.allocs, &sd.w[l], D.w.data(), D.w.size())) ||
        (rc = dev_upload(sd.allocs, &sd.first[l], D.first.data(), D.first.size())) ||
        (rc = dev_upload(sd.allocs, &sd.elo[l], elo.data(), elo.size())) ||
        (rc = dev_upload(sd.allocs, &sd.ehi[l], ehi.data(), ehi.size())))
      return rc;
  }
  if (base_interleaved) {
    const size_t n = size_t(hp.N_s) * hp.stencil * 3;
    if (int rc = dev_upload(sd.allocs, &sd.base, base_interleaved, n)) return rc;
  }
  return 0;
}

void spatial_device_free(SpatialDevice& sd) {
  for (double* a : sd.arrays) (void)hipFree(a);
  sd.arrays.clear();
  for (void* p : sd.allocs) (void)hipFree(p);
  sd.allocs.clear();
}

int spatial_device_apply(const HostProblem& hp, const SpatialModel& m, SpatialDevice& sd, double* Sc_dev,
                         hipStream_t stream) {
  // (re)upload the coefficient arrays
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return int(e);
  for (double* a : sd.arrays) (void)hipFree(a);
  sd.arrays.clear();
  for (const std::vector<double>& a : m.arrays) {
    double* p = nullptr;
    e = hipMalloc(reinterpret_cast<void**>(&p), std::max<size_t>(a.size(), 1) * sizeof(double));
    if (e != hipSuccess) return int(e);
    sd.arrays.push_back(p);
    e = hipMemcpy(p, a.data(), a.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return int(e);
  }
  const int64_t ns = hp.N_s * hp.stencil;
  if (!Sc_dev) return 0;  // coefficient arrays only (the sum-factorised matvec has no stencils)
  if (hp.d > 2) {
    // three directions: sum-factorised host quadrature, then upload (layout [N_s][stencil][3])
    std::vector<double> S(hp.Sc);
    if (m.kronecker_base == false) std::fill(S.begin(), S.end(), 0.0);
    apply_terms_host(hp, m, S.data());
    std::vector<double> I(size_t(ns) * 3);
    for (int64_t k = 0; k < ns; ++k)
      for (int c = 0; c < 3; ++c) I[size_t(k) * 3 + c] = S[size_t(c) * ns + k];
    e = hipMemcpy(Sc_dev, I.data(), I.size() * sizeof(double), hipMemcpyHostToDevice);
    return int(e);
  }
  if (m.terms.size() > size_t(kMaxWTerms)) return int(hipErrorInvalidValue);
  WTermList L;
  L.count = int(m.terms.size());
  for (int k = 0; k < L.count; ++k) {
    const WeightedTerm& t = m.terms[size_t(k)];
    L.t[k].cq = t.coef >= 0 ? sd.arrays[size_t(t.coef)] : nullptr;
    for (int l = 0; l < 2; ++l) {
      L.t[k].a[l] = t.a[l];
      L.t[k].b[l] = t.b[l];
    }
    L.t[k].scale = t.scale;
    L.t[k].target = t.target;
  }
  SpatialTables T;
  for (int l = 0; l < 2; ++l) {
    T.B[l] = sd.B[l];
    T.w[l] = sd.w[l];
    T.first[l] = sd.first[l];
    T.elo[l] = sd.elo[l];
    T.ehi[l] = sd.ehi[l];
    T.Q[l] = l < hp.d ? int(hp.dir_s[l].x.size()) : 1;
  }
  const int blocks = int((ns + 255) / 256);
  hipLaunchKernelGGL(weighted_stencil_kernel, dim3(blocks), dim3(256), 0, stream, L, T,
                     (const double*)(m.kronecker_base ? sd.base : nullptr), Sc_dev, hp.d, hp.n_s[0],
                     hp.d > 1 ? hp.n_s[1] : 1, hp.N_s, hp.stencil, hp.p_s, hp.dir_s[0].q);
  return int(hipGetLastError());
}

}  // namespace stfd
