// Weighted-term model of the spatial factors (unit cube or quarter annulus).
#include "spatial.h"

#include <cmath>

namespace stfd {

namespace {

// Quarter circle as a rational quadratic arc: control points (1,0), (1,1), (0,1), weights
// 1, sqrt(2)/2, 1 (exact circle).  Returns c(t), c'(t), c''(t).
void arc(double t, double c[2], double c1[2], double c2[2]) {
  const double w1 = std::sqrt(0.5);
  const double u = 1.0 - t;
  const double N[2] = {u * u + 2.0 * t * u * w1, 2.0 * t * u * w1 + t * t};
  const double N1[2] = {-2.0 * u + 2.0 * w1 * (1.0 - 2.0 * t), 2.0 * w1 * (1.0 - 2.0 * t) + 2.0 * t};
  const double N2[2] = {2.0 - 4.0 * w1, 2.0 - 4.0 * w1};
  const double W = u * u + 2.0 * t * u * w1 + t * t;
  const double W1 = -2.0 * u + 2.0 * w1 * (1.0 - 2.0 * t) + 2.0 * t;
  const double W2 = 4.0 - 4.0 * w1;
  for (int k = 0; k < 2; ++k) {
    c[k] = N[k] / W;
    const double num = N1[k] * W - N[k] * W1;
    c1[k] = num / (W * W);
    c2[k] = (N2[k] * W - N[k] * W2) / (W * W) - 2.0 * W1 * num / (W * W * W);
  }
}

}  // namespace

void map_points(const Geometry& g, int d, const double* xi, int64_t n, double* x) {
  for (int64_t k = 0; k < n; ++k) {
    if (g.kind == GEOM_QUARTER_ANNULUS && d == 2) {
      double c[2], c1[2], c2[2];
      arc(xi[2 * k + 1], c, c1, c2);
      const double r = g.r0 + (g.r1 - g.r0) * xi[2 * k];
      x[2 * k] = r * c[0];
      x[2 * k + 1] = r * c[1];
    } else {
      for (int l = 0; l < d; ++l) x[d * k + l] = xi[d * k + l];
    }
  }
}

int build_spatial_model(const HostProblem& hp, const Geometry& g, const double* V_quad, SpatialModel& m) {
  const int d = hp.d;
  const double nu = hp.nu;
  int Q[3] = {1, 1, 1};
  size_t nq = 1;
  for (int l = 0; l < d; ++l) {
    Q[l] = int(hp.dir_s[l].x.size());
    nq *= size_t(Q[l]);
  }
  m = SpatialModel();
  auto add_array = [&](std::vector<double> a) {
    m.arrays.push_back(std::move(a));
    return int(m.arrays.size()) - 1;
  };
  auto add_term = [&](int coef, const int* a, const int* b, double scale, int target) {
    WeightedTerm t;
    t.coef = coef;
    for (int l = 0; l < 3; ++l) {
      t.a[l] = a ? a[l] : 0;
      t.b[l] = b ? b[l] : 0;
    }
    t.scale = scale;
    t.target = target;
    m.terms.push_back(t);
  };
  if (V_quad) {
    for (size_t k = 0; k < nq; ++k)
      if (!std::isfinite(V_quad[k])) return -1;
    m.V = add_array(std::vector<double>(V_quad, V_quad + nq));
  }
  if (g.kind == GEOM_UNIT) {
    m.kronecker_base = true;
    for (int l = 0; l < d; ++l) {
      LapTerm t;
      t.ord[l] = 2;
      m.lap.push_back(t);
    }
    if (m.V >= 0) {
      const std::vector<double>& V = m.arrays[size_t(m.V)];
      std::vector<double> V2(nq);
      for (size_t k = 0; k < nq; ++k) V2[k] = V[k] * V[k];
      const int iv2 = add_array(std::move(V2));
      add_term(m.V, nullptr, nullptr, 1.0, 2);  // S_3 += M_V
      add_term(iv2, nullptr, nullptr, 1.0, 1);  // S_2 += M_{V^2}
      for (int l = 0; l < d; ++l) {             // S_2 -= nu (K_V + K_V^T), K_V = int V phi_I d_l^2 phi_J
        int two[3] = {0, 0, 0};
        two[l] = 2;
        add_term(m.V, nullptr, two, -nu, 1);
        add_term(m.V, two, nullptr, -nu, 1);
      }
    }
    return 0;
  }
  if (g.kind != GEOM_QUARTER_ANNULUS || d != 2 || !(g.r0 > 0.0) || !(g.r1 > g.r0)) return -1;
  // orthogonal coordinates (rho, theta): h_rho = dr, h_theta = r s(theta), J = dr r s,
  // Lap u = u_rr / dr^2 + u_r / (dr r) + u_tt / (r s)^2 - s' u_t / (r^2 s^3)
  m.kronecker_base = false;
  const double dr = g.r1 - g.r0;
  std::vector<double> J(nq), cr2(nq), cr1(nq), ct2(nq), ct1(nq), grr(nq), gtt(nq);
  for (int i2 = 0; i2 < Q[1]; ++i2) {
    double c[2], c1[2], c2[2];
    arc(hp.dir_s[1].x[size_t(i2)], c, c1, c2);
    const double s = c[0] * c1[1] - c[1] * c1[0];   // d(angle)/dtheta
    const double s1 = c[0] * c2[1] - c[1] * c2[0];  // its derivative
    for (int i1 = 0; i1 < Q[0]; ++i1) {
      const double r = g.r0 + dr * hp.dir_s[0].x[size_t(i1)];
      const size_t k = size_t(i2) * Q[0] + i1;
      J[k] = dr * r * s;
      cr2[k] = 1.0 / (dr * dr);
      cr1[k] = 1.0 / (dr * r);
      ct2[k] = 1.0 / (r * r * s * s);
      ct1[k] = -s1 / (r * r * s * s * s);
      grr[k] = r * s / dr;   // J / h_rho^2
      gtt[k] = dr / (r * s);  // J / h_theta^2
    }
  }
  m.J = add_array(J);
  const int ord[4][3] = {{2, 0, 0}, {1, 0, 0}, {0, 2, 0}, {0, 1, 0}};
  std::vector<double>* cf[4] = {&cr2, &cr1, &ct2, &ct1};
  int ic[4], icJ[4];
  for (int k = 0; k < 4; ++k) {
    std::vector<double> cj(nq);
    for (size_t q = 0; q < nq; ++q) cj[q] = (*cf[k])[q] * J[q];
    ic[k] = add_array(*cf[k]);
    icJ[k] = add_array(std::move(cj));
    LapTerm t;
    for (int l = 0; l < 3; ++l) t.ord[l] = ord[k][l];
    t.coef = ic[k];
    t.coefJ = icJ[k];
    m.lap.push_back(t);
  }
  // S_1 = int phi phi J
  add_term(m.J, nullptr, nullptr, 1.0, 0);
  // S_3 = nu int grad . grad + M_V
  {
    const int a1[3] = {1, 0, 0}, a2[3] = {0, 1, 0};
    add_term(add_array(grr), a1, a1, nu, 2);
    add_term(add_array(gtt), a2, a2, nu, 2);
  }
  // S_2 = nu^2 int Lap phi_I Lap phi_J J
  for (int k = 0; k < 4; ++k)
    for (int l = 0; l < 4; ++l) {
      std::vector<double> w(nq);
      for (size_t q = 0; q < nq; ++q) w[q] = (*cf[k])[q] * (*cf[l])[q] * J[q];
      add_term(add_array(std::move(w)), ord[k], ord[l], nu * nu, 1);
    }
  if (m.V >= 0) {
    const std::vector<double> V = m.arrays[size_t(m.V)];
    std::vector<double> VJ(nq), V2J(nq);
    for (size_t q = 0; q < nq; ++q) {
      VJ[q] = V[q] * J[q];
      V2J[q] = V[q] * V[q] * J[q];
    }
    add_term(add_array(std::move(VJ)), nullptr, nullptr, 1.0, 2);
    add_term(add_array(std::move(V2J)), nullptr, nullptr, 1.0, 1);
    for (int k = 0; k < 4; ++k) {  // -nu (K_V + K_V^T), K_V = int V phi_I Lap phi_J J
      std::vector<double> w(nq);
      for (size_t q = 0; q < nq; ++q) w[q] = V[q] * m.arrays[size_t(icJ[k])][q];
      const int iw = add_array(std::move(w));
      add_term(iw, nullptr, ord[k], -nu, 1);
      add_term(iw, ord[k], nullptr, -nu, 1);
    }
  }
  return 0;
}

namespace {

// Dirichlet-reduced weighted 1D Gram matrix out[i][j] = int w b_i^(r) b_j^(r) (element Gauss rule).
template <typename Wf>
void weighted_gram_1d(const Direction& D, int r, Wf w, std::vector<double>& out) {
  const int n = D.m - 2;
  out.assign(size_t(n) * n, 0.0);
  for (int e = 0; e < D.n_el; ++e)
    for (int g = 0; g < D.q; ++g) {
      const size_t q = size_t(e) * D.q + g;
      const double wq = D.w[q] * w(D.x[q]);
      for (int a = 0; a <= D.p; ++a) {
        const int i = D.first[e] + a - 1;
        if (i < 0 || i >= n) continue;
        for (int b = 0; b <= D.p; ++b) {
          const int j = D.first[e] + b - 1;
          if (j < 0 || j >= n) continue;
          out[size_t(i) * n + j] += wq * D.b(e, g, r, a) * D.b(e, g, r, b);
        }
      }
    }
}

}  // namespace

int geometry_pencils(HostProblem& hp, const Geometry& g) {
  if (g.kind != GEOM_QUARTER_ANNULUS || hp.d != 2) return -1;
  const double r0 = g.r0, dr = g.r1 - g.r0;
  const Direction& Dr = hp.dir_s[0];
  const Direction& Dt = hp.dir_s[1];
  const int nr = hp.n_s[0], nth = hp.n_s[1];
  auto s_of = [](double t) {
    double c[2], c1[2], c2[2];
    arc(t, c, c1, c2);
    return c[0] * c1[1] - c[1] * c1[0];
  };
  // theta pencil: stiffness weight 1/s, mass weight s
  std::vector<double> Kt, Mt;
  weighted_gram_1d(Dt, 1, [&](double t) { return 1.0 / s_of(t); }, Kt);
  weighted_gram_1d(Dt, 0, [&](double t) { return s_of(t); }, Mt);
  std::vector<double> V(static_cast<size_t>(nth) * nth), mu(static_cast<size_t>(nth));
  if (gen_eig(nth, Kt.data(), Mt.data(), V.data(), mu.data())) return -2;
  // rho pencils: stiffness weight r/dr, cross weight dr/r, mass weight dr r
  std::vector<double> Kr, Xr, Mr;
  weighted_gram_1d(Dr, 1, [&](double x) { return (r0 + dr * x) / dr; }, Kr);
  weighted_gram_1d(Dr, 0, [&](double x) { return dr / (r0 + dr * x); }, Xr);
  weighted_gram_1d(Dr, 0, [&](double x) { return dr * (r0 + dr * x); }, Mr);
  hp.Uslice.assign(size_t(nth) * nr * nr, 0.0);
  hp.lam.assign(size_t(nr) * nth, 0.0);
  std::vector<double> A(static_cast<size_t>(nr) * nr), W(static_cast<size_t>(nr) * nr), lam(static_cast<size_t>(nr));
  for (int j = 0; j < nth; ++j) {
    for (size_t k = 0; k < A.size(); ++k) A[k] = Kr[k] + mu[size_t(j)] * Xr[k];
    if (gen_eig(nr, A.data(), Mr.data(), W.data(), lam.data())) return -2;
    std::copy(W.begin(), W.end(), hp.Uslice.begin() + size_t(j) * nr * nr);
    for (int i = 0; i < nr; ++i) hp.lam[size_t(j) * nr + i] = lam[size_t(i)];
  }
  hp.U[1] = V;
  hp.lam1[1] = mu;
  return time_factors(hp);
}

void apply_terms_host(const HostProblem& hp, const SpatialModel& m, double* Sc) {
  const size_t ns = size_t(hp.N_s) * hp.stencil;
  for (const WeightedTerm& t : m.terms) {
    std::vector<double> tmp(ns, 0.0);
    int ders[3][2];
    for (int l = 0; l < 3; ++l) {
      ders[l][0] = t.a[l];
      ders[l][1] = t.b[l];
    }
    weighted_form(hp, t.coef >= 0 ? m.arrays[size_t(t.coef)].data() : nullptr, ders, tmp.data());
    double* out = Sc + size_t(t.target) * ns;
    for (size_t k = 0; k < ns; ++k) out[k] += t.scale * tmp[k];
  }
}

}  // namespace stfd
