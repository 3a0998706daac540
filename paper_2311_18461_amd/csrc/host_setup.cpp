// Host-side FP64 setup of the space-time least-squares system and of the
// fast-diagonalisation preconditioner (Algorithm 1 step 1, eqs. space_mat,
// time_mat, syst_mat, space_eig; potential terms of S_V = i d_t - nu Lap + V).
//
// Runs once per problem; nothing here is on the iteration path.
#include "host_setup.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

namespace stfd {

static constexpr int kMaxDeg = 12;

// ---------------------------------------------------------------------------
// knot vectors (Section 3.1, Assumption 2)
// ---------------------------------------------------------------------------
int validate_knots(const double* kn, int nk, int p, int max_interior_mult) {
  if (!kn || p < 1 || p > kMaxDeg || nk < 2 * (p + 1)) return -1;
  for (int i = 0; i < nk; ++i)
    if (!std::isfinite(kn[i]) || kn[i] < 0.0 || kn[i] > 1.0) return -1;
  for (int i = 1; i < nk; ++i)
    if (kn[i] < kn[i - 1]) return -1;
  // open: first and last p+1 knots equal to 0 and 1, and not more
  for (int i = 0; i <= p; ++i)
    if (kn[i] != 0.0 || kn[nk - 1 - i] != 1.0) return -1;
  if (kn[p + 1] == 0.0 || kn[nk - p - 2] == 1.0) return -1;
  int i = p + 1;
  while (i < nk - p - 1) {
    int j = i;
    while (j + 1 < nk - p - 1 && kn[j + 1] == kn[i]) ++j;
    if (j - i + 1 > max_interior_mult) return -1;
    i = j + 1;
  }
  return 0;
}

// Gauss-Legendre nodes/weights on (-1,1) by Newton's method on P_q with the
// three-term recurrence; weights 2 / ((1 - x^2) P_q'(x)^2).
int gauss_legendre(int q, double* x, double* w) {
  if (q < 1 || q > 64) return -1;
  for (int i = 0; i < (q + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double pk = z, pkm1 = 1.0;
      for (int k = 2; k <= q; ++k) {
        double pn = ((2.0 * k - 1.0) * z * pk - (k - 1.0) * pkm1) / k;
        pkm1 = pk;
        pk = pn;
      }
      // pk = P_q(z), pkm1 = P_{q-1}(z)
      dp = (q == 1) ? 1.0 : q * (z * pk - pkm1) / (z * z - 1.0);
      double dz = pk / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute derivative at the converged node
    double pk = z, pkm1 = 1.0;
    for (int k = 2; k <= q; ++k) {
      double pn = ((2.0 * k - 1.0) * z * pk - (k - 1.0) * pkm1) / k;
      pkm1 = pk;
      pk = pn;
    }
    dp = (q == 1) ? 1.0 : q * (z * pk - pkm1) / (z * z - 1.0);
    x[i] = -z;
    x[q - 1 - i] = z;
    w[i] = w[q - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  return 0;
}

// Non-zero B-splines of degree p at x in knot span `span` (kn[span] <= x < kn[span+1])
// and their derivatives up to order nder.  Triangular table of basis values
// (upper part) and knot differences (lower part), then derivatives as scaled
// differences of lower-degree values (de Boor's derivative formula applied r times).
static void eval_span(const double* kn, int p, int span, double x, int nder, double* out) {
  double left[kMaxDeg + 1], right[kMaxDeg + 1];
  double ndu[kMaxDeg + 1][kMaxDeg + 1];
  double a[2][kMaxDeg + 1];
  ndu[0][0] = 1.0;
  for (int j = 1; j <= p; ++j) {
    left[j] = x - kn[span + 1 - j];
    right[j] = kn[span + j] - x;
    double saved = 0.0;
    for (int r = 0; r < j; ++r) {
      ndu[j][r] = right[r + 1] + left[j - r];
      double tmp = ndu[r][j - 1] / ndu[j][r];
      ndu[r][j] = saved + right[r + 1] * tmp;
      saved = left[j - r] * tmp;
    }
    ndu[j][j] = saved;
  }
  for (int j = 0; j <= p; ++j) out[j] = ndu[j][p];
  for (int k = 1; k <= nder; ++k)
    for (int j = 0; j <= p; ++j) out[k * (p + 1) + j] = 0.0;
  for (int r = 0; r <= p; ++r) {
    int s1 = 0, s2 = 1;
    a[0][0] = 1.0;
    for (int k = 1; k <= nder && k <= p; ++k) {
      double dd = 0.0;
      int rk = r - k, pk = p - k;
      if (r >= k) {
        a[s2][0] = a[s1][0] / ndu[pk + 1][rk];
        dd = a[s2][0] * ndu[rk][pk];
      }
      int j1 = (rk >= -1) ? 1 : -rk;
      int j2 = (r - 1 <= pk) ? k - 1 : p - r;
      for (int j = j1; j <= j2; ++j) {
        a[s2][j] = (a[s1][j] - a[s1][j - 1]) / ndu[pk + 1][rk + j];
        dd += a[s2][j] * ndu[rk + j][pk];
      }
      if (r <= pk) {
        a[s2][k] = -a[s1][k - 1] / ndu[pk + 1][r];
        dd += a[s2][k] * ndu[r][pk];
      }
      out[k * (p + 1) + r] = dd;
      std::swap(s1, s2);
    }
  }
  double fac = p;
  for (int k = 1; k <= nder; ++k) {
    for (int j = 0; j <= p; ++j) out[k * (p + 1) + j] *= fac;
    fac *= (p - k);
  }
}

int build_direction(const double* kn_in, int nk, int p, int q, double scale, Direction& D) {
  D.p = p;
  D.q = q;
  D.m = nk - p - 1;
  D.knots.assign(kn_in, kn_in + nk);
  for (double& k : D.knots) k *= scale;
  std::vector<double> gx(q), gw(q);
  if (gauss_legendre(q, gx.data(), gw.data())) return -1;
  D.first.clear();
  D.x.clear();
  D.w.clear();
  D.basis.clear();
  std::vector<double> tmp(3 * (p + 1));
  for (int s = p; s < nk - p - 1; ++s) {
    double a = D.knots[s], b = D.knots[s + 1];
    if (!(b > a)) continue;
    D.first.push_back(s - p);
    for (int g = 0; g < q; ++g) {
      double x = 0.5 * (a + b) + 0.5 * (b - a) * gx[g];
      D.x.push_back(x);
      D.w.push_back(0.5 * (b - a) * gw[g]);
      eval_span(D.knots.data(), p, s, x, std::min(2, p), tmp.data());
      for (int r = 0; r < 3; ++r)
        for (int i = 0; i <= p; ++i) D.basis.push_back(r <= p ? tmp[r * (p + 1) + i] : 0.0);
    }
  }
  D.n_el = int(D.first.size());
  return D.n_el > 0 ? 0 : -1;
}

void gram_1d(const Direction& D, Gram1D& g) {
  const int m = D.m, p = D.p;
  g.m = m;
  g.M.assign(size_t(m) * m, 0.0);
  g.L.assign(size_t(m) * m, 0.0);
  g.J.assign(size_t(m) * m, 0.0);
  g.G.assign(size_t(m) * m, 0.0);
  for (int e = 0; e < D.n_el; ++e)
    for (int gq = 0; gq < D.q; ++gq) {
      double w = D.w[size_t(e) * D.q + gq];
      for (int a = 0; a <= p; ++a)
        for (int b = 0; b <= p; ++b) {
          size_t ij = size_t(D.first[e] + a) * m + (D.first[e] + b);
          g.M[ij] += w * D.b(e, gq, 0, a) * D.b(e, gq, 0, b);
          g.L[ij] += w * D.b(e, gq, 1, a) * D.b(e, gq, 1, b);
          g.J[ij] += w * D.b(e, gq, 2, a) * D.b(e, gq, 2, b);
          g.G[ij] += w * D.b(e, gq, 0, a) * D.b(e, gq, 1, b);
        }
    }
}

// ---------------------------------------------------------------------------
// generalised symmetric-definite eigenproblem L U = M U Lambda, U^T M U = I
// (eq. space_eig): M = C C^T (Cholesky), C^{-1} L C^{-T} = Q Lambda Q^T by
// cyclic Jacobi rotations, U = C^{-T} Q; eigenvalues ascending.
// ---------------------------------------------------------------------------
int gen_eig(int n, const double* Lm, const double* Mm, double* U, double* lam) {
  std::vector<double> C(size_t(n) * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = Mm[size_t(j) * n + j];
    for (int k = 0; k < j; ++k) s -= C[size_t(j) * n + k] * C[size_t(j) * n + k];
    if (!(s > 0.0)) return -2;
    double cjj = std::sqrt(s);
    C[size_t(j) * n + j] = cjj;
    for (int i = j + 1; i < n; ++i) {
      double t = Mm[size_t(i) * n + j];
      for (int k = 0; k < j; ++k) t -= C[size_t(i) * n + k] * C[size_t(j) * n + k];
      C[size_t(i) * n + j] = t / cjj;
    }
  }
  // X = C^{-1} L (forward substitution per column), A = C^{-1} X^T = C^{-1} L C^{-T}
  std::vector<double> X(size_t(n) * n), A(size_t(n) * n);
  auto lower_solve = [&](const double* rhs_col_major_stride, size_t stride, double* out, size_t ostride) {
    for (int i = 0; i < n; ++i) {
      double s = rhs_col_major_stride[size_t(i) * stride];
      for (int k = 0; k < i; ++k) s -= C[size_t(i) * n + k] * out[size_t(k) * ostride];
      out[size_t(i) * ostride] = s / C[size_t(i) * n + i];
    }
  };
  for (int c = 0; c < n; ++c) lower_solve(Lm + c, n, X.data() + c, n);      // column c of X
  for (int c = 0; c < n; ++c) lower_solve(X.data() + size_t(c) * n, 1, A.data() + c, n);  // uses row c of X = column c of X^T
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) {
      double s = 0.5 * (A[size_t(i) * n + j] + A[size_t(j) * n + i]);
      A[size_t(i) * n + j] = A[size_t(j) * n + i] = s;
    }
  std::vector<double> Q(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) Q[size_t(i) * n + i] = 1.0;
  double scale = 0.0;
  for (size_t i = 0; i < A.size(); ++i) scale = std::max(scale, std::fabs(A[i]));
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off = std::max(off, std::fabs(A[size_t(i) * n + j]));
    if (off <= 1e-17 * scale) break;
    for (int pp = 0; pp < n - 1; ++pp)
      for (int qq = pp + 1; qq < n; ++qq) {
        double apq = A[size_t(pp) * n + qq];
        if (std::fabs(apq) <= 1e-300) continue;
        double app = A[size_t(pp) * n + pp], aqq = A[size_t(qq) * n + qq];
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns pp, qq
          double akp = A[size_t(k) * n + pp], akq = A[size_t(k) * n + qq];
          A[size_t(k) * n + pp] = c * akp - s * akq;
          A[size_t(k) * n + qq] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows pp, qq
          double apk = A[size_t(pp) * n + k], aqk = A[size_t(qq) * n + k];
          A[size_t(pp) * n + k] = c * apk - s * aqk;
          A[size_t(qq) * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double qkp = Q[size_t(k) * n + pp], qkq = Q[size_t(k) * n + qq];
          Q[size_t(k) * n + pp] = c * qkp - s * qkq;
          Q[size_t(k) * n + qq] = s * qkp + c * qkq;
        }
      }
  }
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(),
            [&](int a, int b) { return A[size_t(a) * n + a] < A[size_t(b) * n + b]; });
  // U = C^{-T} Q: back substitution with C^T for each column of Q
  for (int cc = 0; cc < n; ++cc) {
    int src = order[cc];
    lam[cc] = A[size_t(src) * n + src];
    for (int i = n - 1; i >= 0; --i) {
      double s = Q[size_t(i) * n + src];
      for (int k = i + 1; k < n; ++k) s -= C[size_t(k) * n + i] * U[size_t(k) * n + cc];
      U[size_t(i) * n + cc] = s / C[size_t(i) * n + i];
    }
  }
  return 0;
}

// ---------------------------------------------------------------------------
// potential terms: int c(x) phi_I D phi_J by element-wise tensor Gauss
// quadrature, contracted one direction at a time, scattered into stencil rows.
// ders[l] = {order on phi_I, order on phi_J} in direction l.
// ---------------------------------------------------------------------------
void weighted_form(const HostProblem& hp, const double* cq, const int (*ders)[2], double* out_stencil) {
  const int d = hp.d, p = hp.p_s, nl = p + 1, w2 = 2 * p + 1;
  int Q[3] = {1, 1, 1};
  int nel[3] = {1, 1, 1};
  for (int l = 0; l < d; ++l) {
    Q[l] = int(hp.dir_s[l].x.size());
    nel[l] = hp.dir_s[l].n_el;
  }
  const int q = hp.dir_s[0].q;
  int npts = 1;
  for (int l = 0; l < d; ++l) npts *= q;
  // one element: quadrature weights at its points, sum-factorised contraction, scatter into the
  // stencil rows of its basis functions
  auto element = [&](const int (&e)[3], std::vector<double>& cur, std::vector<double>& nxt) {
    // cur[(g_1 q + g_2) q + g_3] = weight at the local points (direction 1 slowest, so
    // that each contraction below removes the slowest remaining point index)
    cur.assign(npts, 0.0);
    for (int g = 0; g < npts; ++g) {
      int gl[3] = {0, 0, 0};
      int rg = g;
      for (int l = d - 1; l >= 0; --l) { gl[l] = rg % q; rg /= q; }
      size_t gi = 0, st = 1;
      for (int l = 0; l < d; ++l) { gi += size_t(e[l] * q + gl[l]) * st; st *= Q[l]; }
      cur[g] = cq ? cq[gi] : 1.0;
    }
    // contract direction l: pairs (a_l, b_l) replace g_l; layout [pairs so far][remaining g]
    int npairs = 1, rem = npts;
    for (int l = 0; l < d; ++l) {
      rem /= q;
      const Direction& D = hp.dir_s[l];
      nxt.assign(size_t(npairs) * nl * nl * rem, 0.0);
      for (int pr = 0; pr < npairs; ++pr)
        for (int a = 0; a < nl; ++a)
          for (int b = 0; b < nl; ++b)
            for (int r = 0; r < rem; ++r) {
              double s = 0.0;
              for (int g = 0; g < q; ++g)
                s += D.w[size_t(e[l]) * q + g] * D.b(e[l], g, ders[l][0], a) * D.b(e[l], g, ders[l][1], b) *
                     cur[(size_t(pr) * q + g) * rem + r];
              nxt[((size_t(pr) * nl + a) * nl + b) * rem + r] = s;
            }
      npairs *= nl * nl;
      cur.swap(nxt);
    }
    // scatter: cur[pairs] with pair index ((a_1 b_1) (a_2 b_2) ...), direction 1 slowest
    for (int pr = 0; pr < npairs; ++pr) {
      int rest = pr;
      int a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
      for (int l = d - 1; l >= 0; --l) {
        b[l] = rest % nl; rest /= nl;
        a[l] = rest % nl; rest /= nl;
      }
      int64_t I = 0, st = 1;
      int s = 0, sst = 1;
      bool ok = true;
      for (int l = 0; l < d; ++l) {
        int ri = hp.dir_s[l].first[e[l]] + a[l] - 1;  // reduced index
        int rj = hp.dir_s[l].first[e[l]] + b[l] - 1;
        if (ri < 0 || ri >= hp.n_s[l] || rj < 0 || rj >= hp.n_s[l]) { ok = false; break; }
        I += int64_t(ri) * st;
        st *= hp.n_s[l];
        s += (rj - ri + p) * sst;
        sst *= w2;
      }
      if (ok) out_stencil[size_t(I) * hp.stencil + s] += cur[pr];
    }
  };
  // threads over the elements of the slowest direction L, one colour e_L mod (p + 1) at a time:
  // elements of one colour share no basis function along L, so their stencil rows are disjoint
  const int L = d - 1, colours = p + 1;
  int nth = int(std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()), 32u));
  nth = std::min(nth, std::max(1, nel[L] / colours));
  auto work = [&](int colour, int tid) {
    std::vector<double> cur, nxt;
    int e[3] = {0, 0, 0};
    for (int eL = colour + tid * colours; eL < nel[L]; eL += nth * colours) {
      e[L] = eL;
      const int n_other = (L >= 1 ? nel[0] : 1) * (L >= 2 ? nel[1] : 1);
      for (int o = 0; o < n_other; ++o) {
        if (L >= 1) e[0] = o % nel[0];
        if (L >= 2) e[1] = o / nel[0];
        element(e, cur, nxt);
      }
    }
  };
  for (int colour = 0; colour < colours; ++colour) {
    if (nth == 1) {
      work(colour, 0);
      continue;
    }
    std::vector<std::thread> pool;
    for (int t = 0; t < nth; ++t) pool.emplace_back(work, colour, t);
    for (std::thread& th : pool) th.join();
  }
}

// LDL^H factors of H_i = L_t + mu^2 M_t + i mu K_t, mu = nu lambda_i (Section 5.2), for the
// current eigenvalues hp.lam.  0 or -2 (a block is not positive definite).
double mean_potential(const HostProblem& hp, const double* V_quad) {
  int64_t Q[3] = {1, 1, 1}, total = 1;
  for (int l = 0; l < hp.d; ++l) {
    Q[l] = int64_t(hp.dir_s[l].w.size());
    total *= Q[l];
  }
  double sw = 0.0, swv = 0.0;
  for (int64_t g = 0; g < total; ++g) {
    int64_t r = g;
    double w = 1.0;
    for (int l = 0; l < hp.d; ++l) {
      w *= hp.dir_s[l].w[size_t(r % Q[l])];
      r /= Q[l];
    }
    sw += w;
    swv += w * V_quad[g];
  }
  return swv / sw;
}

int time_factors(HostProblem& hp) {
  const int pt = hp.p_t, nt = hp.n_t;
  const double nu = hp.nu;
  hp.Lfac.assign(size_t(nt) * pt * hp.N_s, cplx(0.0, 0.0));
  hp.Dinv.assign(size_t(nt) * hp.N_s, 0.0);
  {
    std::vector<cplx> Lrow(size_t(nt) * (pt + 1));  // Lrow[t*(pt+1) + k] = L[t][t-k]
    std::vector<double> D(nt);
    for (int64_t i = 0; i < hp.N_s; ++i) {
      const double mu = nu * hp.lam[i] + hp.shift;
      auto H = [&](int r, int c) -> cplx {
        size_t ix = size_t(r) * nt + c;
        return cplx(hp.Lt[ix] + mu * mu * hp.Mt[ix], mu * hp.Kt[ix]);
      };
      for (int t = 0; t < nt; ++t) {
        for (int k = std::min(pt, t); k >= 1; --k) {
          int j = t - k;
          cplx s = H(t, j);
          for (int kk = k + 1; kk <= std::min(pt, t); ++kk) {  // columns m = t-kk < j
            int mcol = t - kk;
            if (j - mcol > pt) continue;
            s -= Lrow[size_t(t) * (pt + 1) + kk] * D[mcol] * std::conj(Lrow[size_t(j) * (pt + 1) + (j - mcol)]);
          }
          Lrow[size_t(t) * (pt + 1) + k] = s / D[j];
        }
        double dt = H(t, t).real();
        for (int k = 1; k <= std::min(pt, t); ++k) dt -= std::norm(Lrow[size_t(t) * (pt + 1) + k]) * D[t - k];
        if (!(dt > 0.0) || !std::isfinite(dt)) return -2;
        D[t] = dt;
      }
      for (int t = 0; t < nt; ++t) {
        hp.Dinv[size_t(t) * hp.N_s + i] = 1.0 / D[t];
        for (int k = 1; k <= pt; ++k)
          hp.Lfac[(size_t(t) * pt + (k - 1)) * hp.N_s + i] = (t - k >= 0) ? Lrow[size_t(t) * (pt + 1) + k] : cplx(0, 0);
      }
    }
  }
  return 0;
}

// segment lengths compiled per half-bandwidth P (one lane keeps len rows of y, L and 1/D plus two
// P x P transfers in registers)
static const int kSegCand[7][4] = {{0, 0, 0, 0}, {8, 16, 0, 0}, {8, 12, 16, 0}, {6, 8, 12, 16},
                                   {6, 8, 12, 0},  {6, 8, 0, 0},  {6, 0, 0, 0}};

int time_segment_candidates(int n_t, int p_t, int out[4]) {
  if (p_t < 1 || p_t > 6 || n_t < 1) return 0;
  int c = 0;
  for (int len : kSegCand[p_t])
    if (len > 0 && (n_t + len - 1) / len <= 64) out[c++] = len;
  return c;
}

int time_segment_length(int n_t, int p_t) {
  // cost = dependent FP64 work per lane: four sweeps of len rows (4P fused multiply-adds each) and
  // two reduced recurrences of S-1 steps (4P^2 + 4P)
  static const int (&cand)[7][4] = kSegCand;
  if (p_t < 1 || p_t > 6 || n_t < 1) return 0;
  int best = 0;
  double best_cost = 0.0;
  for (int len : cand[p_t]) {
    if (len == 0) continue;
    const int segs = (n_t + len - 1) / len;
    if (segs > 64) continue;
    const double cost = 16.0 * len * p_t + 2.0 * (segs - 1) * (4.0 * p_t * p_t + 4.0 * p_t);
    if (best == 0 || cost < best_cost) {
      best = len;
      best_cost = cost;
    }
  }
  return best;
}

// Lane slots of a plan: slot q = block * mpb + m holds mode slot_mode[q] (-1: empty); without a
// slot list, slot q holds mode q.  Returns the number of blocks, or -1 if the list does not fill
// whole blocks.
static int64_t plan_slots(const HostProblem& hp, int mpb, const std::vector<int64_t>* slot_mode,
                          std::vector<int64_t>& modes) {
  if (slot_mode) {
    if (slot_mode->size() % size_t(mpb) != 0) return -1;
    modes = *slot_mode;
  } else {
    const int64_t nblk = (hp.N_s + mpb - 1) / mpb;
    modes.resize(size_t(nblk * mpb));
    for (int64_t q = 0; q < nblk * mpb; ++q) modes[size_t(q)] = q < hp.N_s ? q : -1;
  }
  return int64_t(modes.size()) / mpb;
}

int time_solve_plan(const HostProblem& hp, int len, bool transfers, TimeSolvePlan& out,
                    const std::vector<int64_t>* slot_mode) {
  const int nt = hp.n_t, P = hp.p_t;
  if (len < P || len < 1) return -1;
  const int segs = (nt + len - 1) / len;
  if (segs > 64) return -1;
  const int mpb = 64 / segs;
  std::vector<int64_t> modes;
  const int64_t nblk = plan_slots(hp, mpb, slot_mode, modes);
  if (nblk < 0) return -1;
  out.len = len;
  out.segs = segs;
  out.mpb = mpb;
  out.blocks = nblk;
  out.Lf.assign(size_t(nblk) * len * P * 64 * 2, 0.0);
  out.Df.assign(size_t(nblk) * len * 64, 0.0);
  out.Tf.assign(transfers ? size_t(nblk) * P * P * 64 * 2 : 0, 0.0);
  out.Tb.assign(transfers ? size_t(nblk) * P * P * 64 * 2 : 0, 0.0);
  // L[t][t-k] of mode i (zero outside the band and for padded rows t >= n_t)
  auto Lv = [&](int64_t i, int t, int k) -> cplx {
    if (t >= nt || t - k < 0) return cplx(0.0, 0.0);
    return hp.Lfac[(size_t(t) * P + (k - 1)) * hp.N_s + i];
  };
  std::vector<cplx> h(P), g(P);
  for (int64_t q = 0; q < nblk * mpb; ++q) {
    const int64_t i = modes[size_t(q)];
    if (i < 0) continue;
    const int64_t b = q / mpb;
    const int m = int(q - b * mpb);
    for (int s = 0; s < segs; ++s) {
      const int lane = m * segs + s, t0 = s * len;
      for (int j = 0; j < len; ++j) {
        const int t = t0 + j;
        if (t < nt) out.Df[(size_t(b) * len + j) * 64 + lane] = hp.Dinv[size_t(t) * hp.N_s + i];
        for (int k = 1; k <= P; ++k) {
          const cplx v = Lv(i, t, k);
          const size_t o = ((((size_t(b) * len + j) * P + (k - 1)) * 64) + lane) * 2;
          out.Lf[o] = v.real();
          out.Lf[o + 1] = v.imag();
        }
      }
      if (!transfers) continue;
      // forward transfer: last P values z_{t0+len-1-a} of the homogeneous forward recurrence
      // over the segment, started from the history z_{t0-1-c} = delta(c, col)
      for (int col = 0; col < P; ++col) {
        std::fill(h.begin(), h.end(), cplx(0.0, 0.0));
        h[col] = 1.0;
        for (int j = 0; j < len; ++j) {
          const int t = t0 + j;
          cplx z(0.0, 0.0);
          for (int k = 1; k <= P; ++k) z -= Lv(i, t, k) * h[k - 1];
          for (int k = P - 1; k >= 1; --k) h[k] = h[k - 1];
          h[0] = z;
        }
        for (int a = 0; a < P; ++a) {
          const size_t o = ((((size_t(b) * P + a) * P + col) * 64) + lane) * 2;
          out.Tf[o] = h[a].real();
          out.Tf[o + 1] = h[a].imag();
        }
      }
      // backward transfer: first P values x_{t0+a} of the homogeneous backward recurrence
      // x_t = -sum_k conj(L[t+k][t]) x_{t+k} over the segment, started from x_{t0+len+c} = delta(c, col)
      for (int col = 0; col < P; ++col) {
        std::fill(g.begin(), g.end(), cplx(0.0, 0.0));
        g[col] = 1.0;
        for (int j = len - 1; j >= 0; --j) {
          const int t = t0 + j;
          cplx x(0.0, 0.0);
          for (int k = 1; k <= P; ++k) x -= std::conj(Lv(i, t + k, k)) * g[k - 1];
          for (int k = P - 1; k >= 1; --k) g[k] = g[k - 1];
          g[0] = x;
        }
        for (int a = 0; a < P; ++a) {
          const size_t o = ((((size_t(b) * P + a) * P + col) * 64) + lane) * 2;
          out.Tb[o] = g[a].real();
          out.Tb[o + 1] = g[a].imag();
        }
      }
    }
  }
  return 0;
}

int time_solve_state_plan(const HostProblem& hp, int len, TimeSolvePlan& out,
                          const std::vector<int64_t>* slot_mode) {
  const int nt = hp.n_t, P = hp.p_t;
  if (len < P || len < 1) return -1;
  const int segs = (nt + len - 1) / len;
  if (segs > 64) return -1;
  const int mpb = 64 / segs;
  std::vector<int64_t> modes;
  const int64_t nblk = plan_slots(hp, mpb, slot_mode, modes);
  if (nblk < 0) return -1;
  out.len = len;
  out.segs = segs;
  out.mpb = mpb;
  out.blocks = nblk;
  out.Lf.clear();
  out.Df.clear();
  out.Tf.clear();
  out.Tb.clear();
  out.Sf.assign(size_t(nblk) * P * P * 64, 0.0);
  const int rows = segs * len;
  out.Hb.assign(size_t(rows) * (P + 1) * 3, 0.0);
  for (int t = 0; t < nt; ++t)
    for (int k = 0; k <= P && k <= t; ++k) {
      const size_t ix = size_t(t) * nt + (t - k), o = (size_t(t) * (P + 1) + k) * 3;
      out.Hb[o] = hp.Lt[ix];
      out.Hb[o + 1] = hp.Mt[ix];
      out.Hb[o + 2] = hp.Kt[ix];
    }
  out.mu.resize(size_t(hp.N_s));
  for (int64_t i = 0; i < hp.N_s; ++i) out.mu[size_t(i)] = hp.nu * hp.lam[size_t(i)] + hp.shift;
  for (int64_t qs = 0; qs < nblk * mpb; ++qs) {
    const int64_t i = modes[size_t(qs)];
    if (i < 0) continue;
    const int64_t b = qs / mpb;
    const int m = int(qs - b * mpb);
    for (int s = 0; s < segs; ++s) {
      const int lane = m * segs + s, t0 = s * len;
      int q = 0;
      auto put = [&](double v) { out.Sf[(size_t(b) * P * P + q++) * 64 + lane] = v; };
      for (int a = 1; a <= P; ++a)
        for (int k = 1; k <= P - a; ++k) {
          const int t = t0 - a;
          cplx v(0.0, 0.0);
          if (t >= 0 && t - k >= 0 && t < nt) v = hp.Lfac[(size_t(t) * P + (k - 1)) * hp.N_s + i];
          put(v.real());
          put(v.imag());
        }
      for (int a = 1; a <= P; ++a) {
        const int t = t0 - a;
        put(t >= 0 && t < nt ? 1.0 / hp.Dinv[size_t(t) * hp.N_s + i] : 1.0);
      }
    }
  }
  return 0;
}

int host_setup(const stfd_setup_desc_view& v, HostProblem& hp) {
  if (v.d < 1 || v.d > 3 || v.p_t < 1 || v.p_s < 2 || v.p_t > kMaxDeg || v.p_s > kMaxDeg) return -1;
  if (!(v.T > 0.0) || !(v.nu > 0.0) || !std::isfinite(v.T) || !std::isfinite(v.nu)) return -1;
  if (v.n_quad < 0 || v.n_quad > 32) return -1;
  if (validate_knots(v.knots_t, v.n_knots_t, v.p_t, v.p_t)) return -1;
  for (int l = 0; l < v.d; ++l)
    if (validate_knots(v.knots_s[l], v.n_knots_s[l], v.p_s, v.p_s - 1)) return -1;
  hp.d = v.d;
  hp.p_t = v.p_t;
  hp.p_s = v.p_s;
  hp.T = v.T;
  hp.nu = v.nu;
  const double nu = v.nu;
  int qt = v.n_quad ? v.n_quad : v.p_t + 1;
  int qs = v.n_quad ? v.n_quad : v.p_s + 1;
  if (build_direction(v.knots_t, v.n_knots_t, v.p_t, qt, v.T, hp.dir_t)) return -1;
  for (int l = 0; l < v.d; ++l)
    if (build_direction(v.knots_s[l], v.n_knots_s[l], v.p_s, qs, 1.0, hp.dir_s[l])) return -1;

  // time (Section 3.2: drop the first function; eq. time_mat); the ultraweak method of Section
  // 4.4 drops the last one (final condition of the test space)
  Gram1D gt;
  gram_1d(hp.dir_t, gt);
  hp.Mfull_t = gt.M;
  hp.time_final = v.time_final;
  const int mt = gt.m, nt = mt - 1, t_off = v.time_final ? 0 : 1;
  hp.n_t = nt;
  hp.Mt.assign(size_t(nt) * nt, 0.0);
  hp.Lt.assign(size_t(nt) * nt, 0.0);
  hp.Kt.assign(size_t(nt) * nt, 0.0);
  for (int i = 0; i < nt; ++i)
    for (int j = 0; j < nt; ++j) {
      size_t f = size_t(i + t_off) * mt + (j + t_off), fT = size_t(j + t_off) * mt + (i + t_off);
      hp.Mt[size_t(i) * nt + j] = gt.M[f];
      hp.Lt[size_t(i) * nt + j] = gt.L[f];
      hp.Kt[size_t(i) * nt + j] = gt.G[f] - gt.G[fT];  // W_t + W_t^* = i (G - G^T)
    }
  // space (drop first and last function per direction)
  hp.N_s = 1;
  for (int l = 0; l < v.d; ++l) {
    Gram1D g;
    gram_1d(hp.dir_s[l], g);
    hp.Mfull_s[l] = g.M;
    const int m = g.m, n = m - 2;
    if (n < 1) return -1;
    hp.n_s[l] = n;
    hp.N_s *= n;
    hp.Ms1[l].resize(size_t(n) * n);
    hp.Ls1[l].resize(size_t(n) * n);
    hp.Js1[l].resize(size_t(n) * n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        size_t f = size_t(i + 1) * m + (j + 1);
        hp.Ms1[l][size_t(i) * n + j] = g.M[f];
        hp.Ls1[l][size_t(i) * n + j] = g.L[f];
        hp.Js1[l][size_t(i) * n + j] = g.J[f];
      }
    hp.U[l].resize(size_t(n) * n);
    hp.lam1[l].resize(n);
    if (gen_eig(n, hp.Ls1[l].data(), hp.Ms1[l].data(), hp.U[l].data(), hp.lam1[l].data())) return -2;
  }
  hp.N = hp.N_s * nt;
  // Kronecker-sum eigenvalues lambda_i = sum_l lambda_{l, i_l}, x_1 fastest
  hp.lam.assign(hp.N_s, 0.0);
  for (int64_t i = 0; i < hp.N_s; ++i) {
    int64_t r = i;
    double s = 0.0;
    for (int l = 0; l < v.d; ++l) {
      s += hp.lam1[l][r % hp.n_s[l]];
      r /= hp.n_s[l];
    }
    hp.lam[i] = s;
  }
  if (int rc = time_factors(hp)) return rc;
  const int pt = v.p_t;
  // time bands of the system factors T_1 = L_t, T_2 = M_t, T_3 = i K_t
  const int wt = 2 * pt + 1;
  hp.Tband.assign(size_t(3) * nt * wt, 0.0);
  for (int t = 0; t < nt; ++t)
    for (int dt = -pt; dt <= pt; ++dt) {
      int j = t + dt;
      if (j < 0 || j >= nt) continue;
      size_t ix = size_t(t) * nt + j;
      hp.Tband[(size_t(0) * nt + t) * wt + dt + pt] = hp.Lt[ix];
      hp.Tband[(size_t(1) * nt + t) * wt + dt + pt] = hp.Mt[ix];
      hp.Tband[(size_t(2) * nt + t) * wt + dt + pt] = hp.Kt[ix];
    }
  int stencil = 1;
  for (int l = 0; l < v.d; ++l) stencil *= 2 * v.p_s + 1;
  hp.stencil = stencil;
  if (v.stencils) base_stencils(hp, v.kronecker_base);
  return 0;
}

// Spatial factors as stencils.  V = 0 part on the unit cube from the 1D matrices
// (on a mapped domain every part comes from weighted terms, added later):
//   S_1 = (x) M_l, S_3 = nu sum_l (L_l in slot l, M elsewhere),
//   S_2 = nu^2 B_s, B_s = sum_l (J_l in slot l) + sum_{l != k} (L_l, L_k in slots l, k)
//   (integration by parts on the Dirichlet-reduced basis).
void base_stencils(HostProblem& hp, bool kronecker_base) {
  const int d = hp.d, ps = hp.p_s, w2 = 2 * ps + 1;
  const double nu = hp.nu;
  const int stencil = hp.stencil;
  hp.Sc.assign(size_t(3) * hp.N_s * stencil, 0.0);
  double* S1 = hp.Sc.data();
  double* S2 = S1 + size_t(hp.N_s) * stencil;
  double* S3 = S2 + size_t(hp.N_s) * stencil;
  for (int64_t i = 0; i < (kronecker_base ? hp.N_s : 0); ++i) {
    int il[3] = {0, 0, 0};
    int64_t r = i;
    for (int l = 0; l < d; ++l) { il[l] = int(r % hp.n_s[l]); r /= hp.n_s[l]; }
    for (int s = 0; s < stencil; ++s) {
      int o[3] = {0, 0, 0};
      int rs = s;
      bool ok = true;
      for (int l = 0; l < d; ++l) {
        o[l] = rs % w2 - ps;
        rs /= w2;
        int j = il[l] + o[l];
        if (j < 0 || j >= hp.n_s[l]) ok = false;
      }
      if (!ok) continue;
      double Mv[3], Lv[3], Jv[3];
      for (int l = 0; l < d; ++l) {
        size_t ix = size_t(il[l]) * hp.n_s[l] + (il[l] + o[l]);
        Mv[l] = hp.Ms1[l][ix];
        Lv[l] = hp.Ls1[l][ix];
        Jv[l] = hp.Js1[l][ix];
      }
      double m_all = 1.0, lsum = 0.0, bsum = 0.0;
      for (int l = 0; l < d; ++l) m_all *= Mv[l];
      for (int l = 0; l < d; ++l) {
        double pl = Lv[l], pj = Jv[l];
        for (int k = 0; k < d; ++k)
          if (k != l) { pl *= Mv[k]; pj *= Mv[k]; }
        lsum += pl;
        bsum += pj;
        for (int k = 0; k < d; ++k) {
          if (k == l) continue;
          double c = Lv[l] * Lv[k];
          for (int o2 = 0; o2 < d; ++o2)
            if (o2 != l && o2 != k) c *= Mv[o2];
          bsum += c;
        }
      }
      size_t ix = size_t(i) * stencil + s;
      S1[ix] = m_all;
      S2[ix] = nu * nu * bsum;
      S3[ix] = nu * lsum;
    }
  }
}

}  // namespace stfd
