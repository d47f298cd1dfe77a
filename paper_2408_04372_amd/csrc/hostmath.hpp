// Host-side numerics of the set-up phase: 1D node sets, quadrature, Lagrange
// bases, temporal matrices of dG(k)/cGP(k) and small dense linear algebra.
#pragma once

#include <cstddef>
#include <vector>

namespace stmg {
namespace hm {

using Vec = std::vector<double>;

// Dense row-major matrix of small size.
struct Mat {
  int r = 0, c = 0;
  Vec a;
  Mat() = default;
  Mat(int r_, int c_) : r(r_), c(c_), a((size_t)r_ * c_, 0.0) {}
  double& operator()(int i, int j) { return a[(size_t)i * c + j]; }
  double operator()(int i, int j) const { return a[(size_t)i * c + j]; }
};

Mat matmul(const Mat& A, const Mat& B);
Mat inverse(const Mat& A);            // Gauss-Jordan with partial pivoting; throws if singular
// A Q = M Q diag(lam) with Q^T M Q = I, for symmetric A and symmetric positive definite M
// (small n): Cholesky of M, then cyclic Jacobi rotations on L^{-1} A L^{-T}.
void sym_gen_eig(const Mat& A, const Mat& M, Mat& Q, Vec& lam);

// n-point Gauss-Legendre rule on [0, 1].
void gauss(int n, Vec& x, Vec& w);
// n-point Gauss-Lobatto points on [0, 1] (n >= 2).
Vec gauss_lobatto(int n);
// n-point Gauss-Radau points on [0, 1] containing t = 1.
Vec gauss_radau_right(int n);
// Lagrange basis on `nodes`: val[q][i] = l_i(x_q), der[q][i] = l_i'(x_q).
void lagrange(const Vec& nodes, const Vec& x, Mat& val, Mat& der);

// Slab-level temporal data (Sections 2.1-2.2).
struct Temporal {
  int n_t = 0, nt_cell = 0, c = 0;
  int method = 0, k = 0;
  double tau = 0.0;
  Mat M_T, A_T, N_T;      // n_t x n_t
  Mat M_tau, N_tilde;     // diagonal blocks (ASM local temporal factors)
  Vec alpha, beta;        // coupling of the first time cell to u0 (alpha) and, for cGP, v0 / F0 (beta)
};
// problem: 0 heat, 1 wave; method: 0 dG, 1 cGP.
Temporal temporal(int problem, int method, int k, int c, double tau);
// Positions in [0, 1] of the temporal DoFs of one time cell (dG: the k+1 right Radau nodes; cGP:
// the last k of the k+1 Gauss-Lobatto nodes).
Vec dof_positions(const Temporal& t);
// Temporal prolongation (fine.n_t x coarse.n_t) between two discretisations of the same slab
// whose coarse trial space lies in the fine one: entry (i, j) is coarse trial function j at
// the time of fine DoF i.  cGP: the first Gauss-Lobatto node of coarse cell M is the last DoF
// of cell M - 1 (in cell 0 it is the slab's initial value, which carries no correction).
Mat temporal_prolongation(const Temporal& fine, const Temporal& coarse);

}  // namespace hm
}  // namespace stmg
