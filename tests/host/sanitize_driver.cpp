// Host setup code under AddressSanitizer and UndefinedBehaviorSanitizer (built by
// tests/test_host_sanitizers.py with g++, no GPU): every host routine of the library on small
// problems (uniform and graded knots, d = 1..3, p = 2..4, both time conditions, with and without a
// potential, the quarter annulus), with plain checks of the results: finite values, the mass
// stencil of the weighted-form assembly equal to the Kronecker-assembled one, the time factors
// reproducing H_i, and every lane slot of the time-solve plans filled exactly once.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_2311_18461_amd/csrc/host_setup.h"
#include "../../paper_2311_18461_amd/csrc/spatial.h"

using namespace stfd;

static int g_fails = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);          \
      ++g_fails;                                                        \
    }                                                                   \
  } while (0)

static bool finite(const std::vector<double>& v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

// open knot vector on [0, 1] with n_el elements, optionally graded towards both ends
static std::vector<double> knots(int n_el, int p, bool graded) {
  std::vector<double> k(size_t(p), 0.0);
  for (int e = 0; e <= n_el; ++e) {
    double x = double(e) / n_el;
    if (graded) x = x * x * (3.0 - 2.0 * x);
    k.push_back(x);
  }
  k.insert(k.end(), size_t(p), 1.0);
  return k;
}

static stfd_setup_desc_view view(int d, int p, const std::vector<double>& kt, const std::vector<double>* ks,
                                 bool kron, bool final_time) {
  stfd_setup_desc_view v{};
  v.d = d;
  v.p_t = p;
  v.p_s = p;
  v.knots_t = kt.data();
  v.n_knots_t = int(kt.size());
  for (int l = 0; l < 3; ++l) {
    v.knots_s[l] = l < d ? ks[l].data() : nullptr;
    v.n_knots_s[l] = l < d ? int(ks[l].size()) : 0;
  }
  v.T = 1.0;
  v.nu = 0.9;
  v.n_quad = 0;
  v.kronecker_base = kron;
  v.stencils = true;
  v.time_final = final_time;
  return v;
}

// H_i = L D L^H rebuilt from the factors of mode i, against L_t + mu^2 M_t + i mu K_t
static double factor_residual(const HostProblem& hp, int64_t i) {
  const int nt = hp.n_t, P = hp.p_t;
  const double mu = hp.nu * hp.lam[size_t(i)] + hp.shift;
  double err = 0.0, scale = 0.0;
  auto L = [&](int r, int c) -> cplx {
    if (r == c) return cplx(1.0, 0.0);
    if (c > r || r - c > P) return cplx(0.0, 0.0);
    return hp.Lfac[(size_t(r) * P + (r - c - 1)) * hp.N_s + i];
  };
  for (int r = 0; r < nt; ++r)
    for (int c = std::max(0, r - P); c <= r; ++c) {
      cplx s(0.0, 0.0);
      for (int k = std::max(0, r - P); k <= c; ++k) s += L(r, k) * (1.0 / hp.Dinv[size_t(k) * hp.N_s + i]) * std::conj(L(c, k));
      const size_t ix = size_t(r) * nt + c;
      const cplx h(hp.Lt[ix] + mu * mu * hp.Mt[ix], mu * hp.Kt[ix]);
      err = std::max(err, std::abs(s - h));
      scale = std::max(scale, std::abs(h));
    }
  return err / scale;
}

static void plans(const HostProblem& hp) {
  int cand[4];
  const int nc = time_segment_candidates(hp.n_t, hp.p_t, cand);
  CHECK(nc > 0 && time_segment_length(hp.n_t, hp.p_t) > 0);
  for (int c = 0; c < nc; ++c)
    for (int form = 0; form < 3; ++form)
      for (int with_slots = 0; with_slots < 2; ++with_slots) {
        const int len = cand[c];
        const int segs = (hp.n_t + len - 1) / len, mpb = 64 / segs;
        // a permuted layout with empty slots: modes in reverse order, one empty slot per block
        std::vector<int64_t> slots;
        if (with_slots) {
          int64_t next = hp.N_s - 1;
          while (next >= 0) {
            for (int m = 0; m < mpb; ++m) slots.push_back(m == mpb - 1 || next < 0 ? -1 : next--);
          }
        }
        TimeSolvePlan tp;
        const std::vector<int64_t>* sl = with_slots ? &slots : nullptr;
        const int rc = form == 2 ? time_solve_state_plan(hp, len, tp, sl) : time_solve_plan(hp, len, form == 0, tp, sl);
        CHECK(rc == 0);
        CHECK(finite(tp.Lf) && finite(tp.Df) && finite(tp.Tf) && finite(tp.Tb) && finite(tp.Sf) && finite(tp.Hb));
        if (form < 2) {
          // every filled slot has positive inverse pivots on its real rows, empty slots none
          const int64_t nslots = tp.blocks * tp.mpb;
          for (int64_t q = 0; q < nslots; ++q) {
            const int64_t mode = with_slots ? slots[size_t(q)] : (q < hp.N_s ? q : -1);
            const int64_t b = q / tp.mpb;
            const int lane = int(q - b * tp.mpb) * tp.segs;
            const double dinv = tp.Df[(size_t(b) * tp.len + 0) * 64 + lane];
            CHECK(mode < 0 ? dinv == 0.0 : dinv > 0.0);
          }
        }
      }
  TimeSolvePlan bad;
  CHECK(time_solve_plan(hp, hp.p_t - 1, true, bad) == -1);  // segments shorter than the band
  const int mpb0 = 64 / ((hp.n_t + cand[0] - 1) / cand[0]);
  if (mpb0 > 1) {
    std::vector<int64_t> ragged(size_t(mpb0 + 1), 0);  // not a whole number of blocks
    CHECK(time_solve_state_plan(hp, cand[0], bad, &ragged) == -1);
    CHECK(time_solve_plan(hp, cand[0], false, bad, &ragged) == -1);
  }
}

static void unit_cube(int d, int p, int n_el, bool graded, bool final_time, bool with_v, std::mt19937_64& rng) {
  const std::vector<double> kt = knots(n_el + 1, p, false);
  std::vector<double> ks[3];
  for (int l = 0; l < d; ++l) ks[l] = knots(n_el + l, p, graded);
  HostProblem hp;
  CHECK(host_setup(view(d, p, kt, ks, true, final_time), hp) == 0);
  CHECK(finite(hp.Mt) && finite(hp.Lt) && finite(hp.Kt) && finite(hp.lam) && finite(hp.Dinv) && finite(hp.Sc));
  CHECK(hp.N == hp.N_s * hp.n_t);
  // the mass stencil of the weighted-form assembly (weight 1, no derivatives) equals S_1 of the
  // Kronecker-assembled base
  std::vector<double> st(size_t(hp.N_s) * hp.stencil, 0.0);
  const int ders[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  weighted_form(hp, nullptr, ders, st.data());
  double dm = 0.0, sm = 0.0;
  for (size_t k = 0; k < st.size(); ++k) {
    dm = std::max(dm, std::abs(st[k] - hp.Sc[k]));
    sm = std::max(sm, std::abs(hp.Sc[k]));
  }
  CHECK(dm <= 1e-13 * sm);
  // potential on the Gauss grid: spatial model, weighted terms, the mean-shifted time factors
  size_t nq = 1;
  for (int l = 0; l < d; ++l) nq *= hp.dir_s[l].x.size();
  std::vector<double> V(nq);
  std::uniform_real_distribution<double> U(0.0, 40.0);
  for (double& x : V) x = U(rng);
  SpatialModel m;
  Geometry g;
  CHECK(build_spatial_model(hp, g, with_v ? V.data() : nullptr, m) == 0);
  std::vector<double> Sc = hp.Sc;
  apply_terms_host(hp, m, Sc.data());
  CHECK(finite(Sc));
  if (with_v) {
    hp.shift = mean_potential(hp, V.data());
    CHECK(std::isfinite(hp.shift) && hp.shift > 0.0 && hp.shift < 40.0);
    CHECK(time_factors(hp) == 0);
  }
  for (int64_t i : {int64_t(0), hp.N_s / 2, hp.N_s - 1}) CHECK(factor_residual(hp, i) < 1e-12);
  plans(hp);
}

static void annulus(int p, int n_el) {
  const std::vector<double> kt = knots(n_el, p, false);
  std::vector<double> ks[3] = {knots(n_el, p, false), knots(n_el + 1, p, false), {}};
  HostProblem hp;
  CHECK(host_setup(view(2, p, kt, ks, false, false), hp) == 0);
  Geometry g;
  g.kind = GEOM_QUARTER_ANNULUS;
  g.r0 = 1.0;
  g.r1 = 2.0;
  SpatialModel m;
  CHECK(build_spatial_model(hp, g, nullptr, m) == 0);
  CHECK(geometry_pencils(hp, g) == 0);
  CHECK(finite(hp.Uslice) && finite(hp.lam) && finite(hp.Dinv));
  std::vector<double> Sc(hp.Sc.size(), 0.0);
  apply_terms_host(hp, m, Sc.data());
  CHECK(finite(Sc));
  const double xi[6] = {0.0, 0.0, 1.0, 1.0, 0.5, 0.25};
  double x[6];
  map_points(g, 2, xi, 3, x);
  for (int k = 0; k < 3; ++k) {
    const double r = std::hypot(x[2 * k], x[2 * k + 1]);
    CHECK(std::abs(r - (1.0 + xi[2 * k])) < 1e-14);  // radius 1 + xi_1 on the whole arc
  }
  plans(hp);
}

static void rejections() {
  const std::vector<double> kt = knots(4, 3, false);
  std::vector<double> ks[3] = {knots(4, 3, false), {}, {}};
  HostProblem hp;
  stfd_setup_desc_view v = view(1, 3, kt, ks, true, false);
  v.p_s = 1;
  CHECK(host_setup(v, hp) == -1);
  std::vector<double> bad = kt;
  std::swap(bad[4], bad[5]);  // decreasing interior knots
  CHECK(validate_knots(bad.data(), int(bad.size()), 3, 3) == -1);
  v = view(1, 3, kt, ks, true, false);
  v.nu = -1.0;
  CHECK(host_setup(v, hp) == -1);
  v = view(1, 3, kt, ks, true, false);
  v.n_quad = 64;
  CHECK(host_setup(v, hp) == -1);
}

int main() {
#if defined(__SANITIZE_ADDRESS__)
  std::printf("address sanitizer: on\n");
#endif
  std::mt19937_64 rng(7);
  for (int p = 2; p <= 4; ++p) {
    unit_cube(1, p, 9, false, false, false, rng);
    unit_cube(1, p, 7, true, true, true, rng);
    unit_cube(2, p, 5, true, false, true, rng);
    unit_cube(2, p, 4, false, true, false, rng);
    unit_cube(3, p, 3, false, false, true, rng);
  }
  annulus(3, 4);
  annulus(4, 3);
  rejections();
  std::printf("%s (%d failed checks)\n", g_fails ? "FAILED" : "OK", g_fails);
  return g_fails ? 1 : 0;
}
