// Host-side setup data of one problem (FP64), shared by host_setup.cpp and stfd.hip.
#pragma once
#include <complex>
#include <cstdint>
#include <vector>

namespace stfd {

using cplx = std::complex<double>;

// One knot vector and its element-wise Gauss rule with basis data.
struct Direction {
  std::vector<double> knots;  // scaled to the physical interval
  int p = 0;
  int m = 0;                  // number of B-splines
  int n_el = 0;               // non-empty spans
  int q = 0;                  // Gauss points per element
  std::vector<int> first;     // first non-zero function on each element
  std::vector<double> x, w;   // n_el * q points and weights
  // basis[((e*q + g)*3 + r)*(p+1) + a]: derivative r of function first[e]+a at point g of element e
  std::vector<double> basis;
  double b(int e, int g, int r, int a) const { return basis[((size_t(e) * q + g) * 3 + r) * (p + 1) + a]; }
};

// Dense full m x m Gram matrices X[i*m+j] = int b_i^(a) b_j^(b).
struct Gram1D {
  int m = 0;
  std::vector<double> M, L, J, G;  // G[i][j] = int b_j' b_i
};

struct HostProblem {
  int d = 0, p_t = 0, p_s = 0;
  double T = 1, nu = 1;
  bool time_final = false;  // time basis without its last function (ultraweak method, Section 4.4)
  double shift = 0.0;       // constant c of the shifted preconditioner: mu_i = nu lambda_i + c
  Direction dir_t;
  Direction dir_s[3];
  int n_t = 0;
  int n_s[3] = {1, 1, 1};
  int64_t N_s = 0, N = 0;
  // reduced 1D matrices
  std::vector<double> Mt, Lt, Kt;  // n_t x n_t; W_t + W_t^* = i Kt
  std::vector<double> Ms1[3], Ls1[3], Js1[3];
  // generalised eigendecomposition per direction: U[j*n + k], lambda[k]
  std::vector<double> U[3], lam1[3];
  std::vector<double> lam;  // eigenvalues of the spatial pencil, N_s (x_1 fastest)
  // Two-level pencils of a mapped domain: direction 0 has one n_0 x n_0 eigenvector
  // matrix per mode of direction 1, Uslice[(j n_0 + r) n_0 + c] (empty: U[0] for all)
  std::vector<double> Uslice;
  // LDL^H factors of H_i, layout [t][k-1][mode] (complex) and [t][mode] (real)
  std::vector<cplx> Lfac;
  std::vector<double> Dinv;
  // time bands T_k[t][dt + p_t], dt = -p_t..p_t  (k = 0: L_t, 1: M_t, 2: K_t)
  std::vector<double> Tband;
  // spatial stencils S_k[i][s], s = sum_l (o_l + p_s) (2p_s+1)^l, k = 0..2
  int stencil = 0;  // (2 p_s + 1)^d
  std::vector<double> Sc;  // 3 * N_s * stencil
  // full (unreduced) 1D mass matrices, for the lifting of initial and boundary data
  std::vector<double> Mfull_t, Mfull_s[3];
};

// Returns 0 or a negative stfd_status.
int validate_knots(const double* kn, int nk, int p, int max_interior_mult);
int build_direction(const double* kn, int nk, int p, int q, double scale, Direction& out);
void gram_1d(const Direction& dir, Gram1D& g);
int gauss_legendre(int q, double* x, double* w);  // on (-1,1)
int gen_eig(int n, const double* L, const double* M, double* U, double* lam);  // 0 or -2
int host_setup(const struct stfd_setup_desc_view& v, HostProblem& hp);
// Mean of the potential samples V_quad (spatial Gauss grid, x_1 fastest) over the unit cube by the
// element Gauss rule of hp.dir_s.
double mean_potential(const HostProblem& hp, const double* V_quad);
// hp.Sc: the V-free unit-cube stencils from the 1D matrices (kronecker_base), else zeros.
void base_stencils(HostProblem& hp, bool kronecker_base);
int time_factors(HostProblem& hp);

// Segmented layout of the banded time solves: each mode's n_t rows are cut into `segs`
// segments of `len` rows (the last padded with zero rows); lane m*segs + s of a 64-lane block
// holds segment s of mode blk*mpb + m.  Tables (doubles, complex as re/im pairs):
//   Lf[blk][j][k-1][lane]  = L[t][t-k], t = s*len + j        (complex)
//   Df[blk][j][lane]       = 1 / D[t]                        (0 on padded rows)
//   Tf[blk][a][c][lane]    = response of z_{t0+len-1-a} to the history z_{t0-1-c}  (complex)
//   Tb[blk][a][c][lane]    = response of x_{t0+a} to the future x_{t0+len+c}        (complex)
// Tf and Tb are built only on request (small grids; large grids compute them in the solve).
// The factor-in-kernel form (large grids) stores no rows of L or 1/D but, per (mode, segment),
// the part of the factor that the rows of the segment depend on:
//   Sf[blk][q][lane], q < P^2: the entries L[t0-a][t0-a-k] (a = 1..P, k = 1..P-a; complex, in
//     that order; zero before t = 0), then D[t0-a] (a = 1..P; 1 before t = 0);
//   Hb[t][k][3] = (L_t, M_t, K_t)[t][t-k] for k = 0..P (zero outside the matrix and past n_t);
//   mu[i] = nu lambda_i, so that H_i[t][t-k] = L_t + mu^2 M_t + i mu K_t.
struct TimeSolvePlan {
  int len = 0, segs = 0, mpb = 0;
  int64_t blocks = 0;
  std::vector<double> Lf, Df, Tf, Tb;
  std::vector<double> Sf, Hb, mu;
};
// State form of the plan (Sf, Hb, mu; no Lf, Df, Tf, Tb).  0, or -1 as time_solve_plan.
int time_solve_state_plan(const HostProblem& hp, int len, TimeSolvePlan& out,
                          const std::vector<int64_t>* slot_mode = nullptr);
// Segment length for n_t rows of half-bandwidth p_t among the compiled ones, 0 if none fits.
int time_segment_length(int n_t, int p_t);
// The compiled segment lengths for half-bandwidth p_t with at most 64 segments (count returned).
int time_segment_candidates(int n_t, int p_t, int out[4]);
// 0, or -1 if len does not fit (len < p_t or more than 64 segments).  slot_mode (optional): the
// mode of every lane slot q = blk * mpb + m (-1 for an empty slot; a whole number of blocks), for
// launches that deal the modes to blocks in another order; by default slot q holds mode q.
int time_solve_plan(const HostProblem& hp, int len, bool transfers, TimeSolvePlan& out,
                    const std::vector<int64_t>* slot_mode = nullptr);
// out_stencil[I][s] += int cq D^{ders[l][0]} phi_I D^{ders[l][1]} phi_J (element Gauss rule, cq on
// the spatial grid or nullptr for 1), for the Dirichlet-reduced spatial basis.
void weighted_form(const HostProblem& hp, const double* cq, const int (*ders)[2], double* out_stencil);

// Flat view of the public descriptor (keeps this header free of the C ABI).
struct stfd_setup_desc_view {
  int d, p_t, p_s;
  const double* knots_t;
  int n_knots_t;
  const double* knots_s[3];
  int n_knots_s[3];
  double T, nu;
  int n_quad;
  bool kronecker_base;  // assemble the V-free unit-cube stencils from 1D matrices
  bool stencils;        // build hp.Sc now (false: the caller decides later)
  bool time_final;      // drop the last time function instead of the first (Section 4.4)
};

}  // namespace stfd
