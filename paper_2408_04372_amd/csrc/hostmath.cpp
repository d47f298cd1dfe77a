// Host numerics of the set-up phase (see hostmath.hpp).
//
// Node sets are computed from Legendre polynomials by bracketing sign changes
// on a fine grid and bisection, which is robust for the small degrees used here.
// Temporal matrices follow Sections 2.1 (dG, right Radau basis, upwind jump) and
// 2.2 (cGP, Gauss-Lobatto trial / last-k test basis), integrated exactly with a
// Gauss rule of sufficient order.
#include "hostmath.hpp"

#include <cmath>
#include <functional>

#include "common.hpp"

namespace stmg {
namespace hm {

Mat matmul(const Mat& A, const Mat& B) {
  Mat C(A.r, B.c);
  for (int i = 0; i < A.r; ++i)
    for (int k = 0; k < A.c; ++k) {
      double a = A(i, k);
      if (a == 0.0) continue;
      for (int j = 0; j < B.c; ++j) C(i, j) += a * B(k, j);
    }
  return C;
}

void sym_gen_eig(const Mat& A, const Mat& M, Mat& Q, Vec& lam) {
  const int n = A.r;
  Mat L(n, n);
  for (int j = 0; j < n; ++j) {
    double d = M(j, j);
    for (int k = 0; k < j; ++k) d -= L(j, k) * L(j, k);
    if (!(d > 0.0)) fail(STMG_E_ARG, "mass matrix of the separable smoother is not positive definite");
    L(j, j) = std::sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double v = M(i, j);
      for (int k = 0; k < j; ++k) v -= L(i, k) * L(j, k);
      L(i, j) = v / L(j, j);
    }
  }
  // C = L^{-1} A L^{-T}: Y = L^{-1} A (column by column), then C = L^{-1} Y^T
  auto lsolve = [&](const Mat& B) {
    Mat X(n, n);
    for (int c = 0; c < n; ++c)
      for (int i = 0; i < n; ++i) {
        double v = B(i, c);
        for (int k = 0; k < i; ++k) v -= L(i, k) * X(k, c);
        X(i, c) = v / L(i, i);
      }
    return X;
  };
  Mat Y = lsolve(A), Yt(n, n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Yt(i, j) = Y(j, i);
  Mat C = lsolve(Yt), V(n, n);
  for (int i = 0; i < n; ++i) V(i, i) = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += C(i, j) * C(i, j);
    if (off < 1e-30) break;
    for (int pq = 0; pq < n * n; ++pq) {
      int p = pq / n, q = pq % n;
      if (q <= p || std::fabs(C(p, q)) < 1e-300) continue;
      double th = (C(q, q) - C(p, p)) / (2.0 * C(p, q));
      double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
      double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
      for (int k = 0; k < n; ++k) {        // C <- G^T C G, V <- V G
        double a = C(k, p), b = C(k, q);
        C(k, p) = c * a - sn * b;
        C(k, q) = sn * a + c * b;
      }
      for (int k = 0; k < n; ++k) {
        double a = C(p, k), b = C(q, k);
        C(p, k) = c * a - sn * b;
        C(q, k) = sn * a + c * b;
      }
      for (int k = 0; k < n; ++k) {
        double a = V(k, p), b = V(k, q);
        V(k, p) = c * a - sn * b;
        V(k, q) = sn * a + c * b;
      }
    }
  }
  lam.assign(n, 0.0);
  for (int i = 0; i < n; ++i) lam[i] = C(i, i);
  // Q = L^{-T} V
  Q = Mat(n, n);
  for (int c = 0; c < n; ++c)
    for (int i = n - 1; i >= 0; --i) {
      double v = V(i, c);
      for (int k = i + 1; k < n; ++k) v -= L(k, i) * Q(k, c);
      Q(i, c) = v / L(i, i);
    }
}

Mat inverse(const Mat& A0) {
  int n = A0.r;
  Mat A = A0, I(n, n);
  for (int i = 0; i < n; ++i) I(i, i) = 1.0;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    double best = std::fabs(A(col, col));
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(A(r, col)) > best) { best = std::fabs(A(r, col)); piv = r; }
    if (best == 0.0 || !std::isfinite(best)) fail(STMG_E_ARG, "singular matrix in set-up");
    if (piv != col)
      for (int j = 0; j < n; ++j) { std::swap(A(col, j), A(piv, j)); std::swap(I(col, j), I(piv, j)); }
    double d = 1.0 / A(col, col);
    for (int j = 0; j < n; ++j) { A(col, j) *= d; I(col, j) *= d; }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      double f = A(r, col);
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) { A(r, j) -= f * A(col, j); I(r, j) -= f * I(col, j); }
    }
  }
  return I;
}

// Legendre P_n and P_n' on [-1, 1] by the three-term recurrence.
static void legendre(int n, double x, double& p, double& dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { p = 1.0; dp = 0.0; return; }
  for (int m = 2; m <= n; ++m) {
    double p2 = ((2.0 * m - 1.0) * x * p1 - (m - 1.0) * p0) / m;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  // derivative from (1 - x^2) P_n' = n (P_{n-1} - x P_n), valid for |x| < 1
  dp = (std::fabs(1.0 - x * x) < 1e-300) ? 0.0 : n * (p0 - x * p1) / (1.0 - x * x);
}

// All roots of f in the open interval (-1, 1) by sign-change bracketing and bisection.
static Vec roots_in(const std::function<double(double)>& f, int expected) {
  Vec out;
  const int M = 20000;
  double xa = -1.0 + 1e-12, fa = f(xa);
  for (int i = 1; i <= M; ++i) {
    double xb = -1.0 + 1e-12 + (2.0 - 2e-12) * i / M;
    double fb = f(xb);
    if (fa == 0.0) { out.push_back(xa); }
    else if (fa * fb < 0.0) {
      double lo = xa, hi = xb, flo = fa;
      for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi), fm = f(mid);
        if (fm == 0.0) { lo = hi = mid; break; }
        if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else { hi = mid; }
      }
      out.push_back(0.5 * (lo + hi));
    }
    xa = xb;
    fa = fb;
  }
  if ((int)out.size() != expected) fail(STMG_E_UNSUPPORTED, "node computation failed");
  return out;
}

void gauss(int n, Vec& x, Vec& w) {
  Vec r = roots_in([n](double t) { double p, dp; legendre(n, t, p, dp); return p; }, n);
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    // polish with Newton and take the weight 2 / ((1 - t^2) P_n'(t)^2)
    double t = r[i];
    for (int it = 0; it < 3; ++it) { double p, dp; legendre(n, t, p, dp); t -= p / dp; }
    double p, dp;
    legendre(n, t, p, dp);
    x[i] = 0.5 * (t + 1.0);
    w[i] = 0.5 * 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

Vec gauss_lobatto(int n) {
  if (n < 2) fail(STMG_E_ARG, "Gauss-Lobatto needs n >= 2");
  Vec out{0.0};
  if (n > 2) {
    Vec r = roots_in([n](double t) { double p, dp; legendre(n - 1, t, p, dp); return dp; }, n - 2);
    for (double t : r) out.push_back(0.5 * (t + 1.0));
  }
  out.push_back(1.0);
  return out;
}

Vec gauss_radau_right(int n) {
  if (n == 1) return Vec{1.0};
  // roots of P_{n-1} - P_n on [-1, 1]; t = 1 is one of them, the other n-1 are interior
  Vec r = roots_in([n](double t) {
    double pa, da, pb, db;
    legendre(n - 1, t, pa, da);
    legendre(n, t, pb, db);
    return pa - pb;
  }, n - 1);
  Vec out;
  for (double t : r) out.push_back(0.5 * (t + 1.0));
  out.push_back(1.0);
  return out;
}

void lagrange(const Vec& nodes, const Vec& x, Mat& val, Mat& der) {
  int n = (int)nodes.size(), m = (int)x.size();
  val = Mat(m, n);
  der = Mat(m, n);
  for (int q = 0; q < m; ++q)
    for (int i = 0; i < n; ++i) {
      double den = 1.0, num = 1.0, dsum = 0.0;
      for (int j = 0; j < n; ++j) {
        if (j == i) continue;
        den *= nodes[i] - nodes[j];
        num *= x[q] - nodes[j];
        double t = 1.0;
        for (int l = 0; l < n; ++l)
          if (l != i && l != j) t *= x[q] - nodes[l];
        dsum += t;
      }
      val(q, i) = num / den;
      der(q, i) = dsum / den;
    }
}

Temporal temporal(int problem, int method, int k, int c, double tau) {
  Temporal T;
  Vec xq, wq;
  gauss(k + 3, xq, wq);
  Mat Mloc, Aloc, sub_M, sub_A;
  int nc;
  if (method == 0) {  // dG(k), right Radau
    Vec nodes = gauss_radau_right(k + 1);
    nc = k + 1;
    Mat V, D, V0, D0;
    lagrange(nodes, xq, V, D);
    lagrange(nodes, Vec{0.0}, V0, D0);
    Mloc = Mat(nc, nc);
    Aloc = Mat(nc, nc);
    for (int i = 0; i < nc; ++i)
      for (int j = 0; j < nc; ++j) {
        double m = 0.0, a = 0.0;
        for (size_t q = 0; q < xq.size(); ++q) {
          m += wq[q] * V(q, i) * V(q, j);
          a += wq[q] * D(q, j) * V(q, i);
        }
        Mloc(i, j) = tau * m;
        Aloc(i, j) = a + V0(0, j) * V0(0, i);   // upwind jump term xi_j(0) xi_i(0)
      }
    sub_M = Mat(nc, nc);
    sub_A = Mat(nc, nc);
    for (int i = 0; i < nc; ++i) sub_A(i, nc - 1) = -V0(0, i);   // -alpha e_N^T
    T.alpha.assign(nc, 0.0);
    T.beta.assign(nc, 0.0);
    for (int i = 0; i < nc; ++i) T.alpha[i] = V0(0, i);
  } else {  // cGP(k): trial at k+1 Gauss-Lobatto points, test at the last k of them
    if (k < 1) fail(STMG_E_ARG, "cGP needs k >= 1");
    Vec trial = gauss_lobatto(k + 1);
    Vec test(trial.begin() + 1, trial.end());
    nc = k;
    Mat Vt, Dt, Vs, Ds;
    lagrange(trial, xq, Vt, Dt);
    lagrange(test, xq, Vs, Ds);
    Mat Mf(nc, k + 1), Af(nc, k + 1);
    for (int i = 0; i < nc; ++i)
      for (int j = 0; j <= k; ++j) {
        double m = 0.0, a = 0.0;
        for (size_t q = 0; q < xq.size(); ++q) {
          m += wq[q] * Vt(q, j) * Vs(q, i);
          a += wq[q] * Dt(q, j) * Vs(q, i);
        }
        Mf(i, j) = tau * m;
        Af(i, j) = a;
      }
    Mloc = Mat(nc, nc);
    Aloc = Mat(nc, nc);
    sub_M = Mat(nc, nc);
    sub_A = Mat(nc, nc);
    for (int i = 0; i < nc; ++i) {
      for (int j = 0; j < nc; ++j) { Mloc(i, j) = Mf(i, j + 1); Aloc(i, j) = Af(i, j + 1); }
      sub_M(i, nc - 1) = Mf(i, 0);   // beta e_N^T: previous cell's last DoF is this cell's first
      sub_A(i, nc - 1) = Af(i, 0);   // alpha e_N^T
    }
    T.alpha.assign(nc, 0.0);
    T.beta.assign(nc, 0.0);
    for (int i = 0; i < nc; ++i) { T.alpha[i] = Af(i, 0); T.beta[i] = Mf(i, 0); }
  }
  int n = nc * c;
  T.n_t = n;
  T.nt_cell = nc;
  T.c = c;
  T.method = method;
  T.k = k;
  T.tau = tau;
  T.M_T = Mat(n, n);
  T.A_T = Mat(n, n);
  for (int m = 0; m < c; ++m)
    for (int i = 0; i < nc; ++i)
      for (int j = 0; j < nc; ++j) {
        T.M_T(m * nc + i, m * nc + j) = Mloc(i, j);
        T.A_T(m * nc + i, m * nc + j) = Aloc(i, j);
        if (m > 0) {
          T.M_T(m * nc + i, (m - 1) * nc + j) = sub_M(i, j);
          T.A_T(m * nc + i, (m - 1) * nc + j) = sub_A(i, j);
        }
      }
  if (problem == 0) T.N_T = T.A_T;
  else T.N_T = matmul(T.A_T, matmul(inverse(T.M_T), T.A_T));
  T.M_tau = Mat(nc, nc);
  T.N_tilde = Mat(nc, nc);
  for (int i = 0; i < nc; ++i)
    for (int j = 0; j < nc; ++j) { T.M_tau(i, j) = T.M_T(i, j); T.N_tilde(i, j) = T.N_T(i, j); }
  // round-off below 1e-15 relative in N_T would only add fill to the sparse row lists
  double mx = 0.0;
  for (double v : T.N_T.a) mx = std::fmax(mx, std::fabs(v));
  for (double& v : T.N_T.a) if (std::fabs(v) < 1e-15 * mx) v = 0.0;
  return T;
}

// local DoF positions in [0, 1] of one time cell: dG the k+1 right Radau nodes, cGP the last
// k of the k+1 Gauss-Lobatto nodes
Vec dof_positions(const Temporal& t) {
  if (t.method == 0) return gauss_radau_right(t.k + 1);
  Vec gl = gauss_lobatto(t.k + 1);
  return Vec(gl.begin() + 1, gl.end());
}

Mat temporal_prolongation(const Temporal& fine, const Temporal& coarse) {
  if (fine.method != coarse.method) fail(STMG_E_ARG, "temporal transfer between different methods");
  const Vec fpos = dof_positions(fine);
  const Vec cnodes = coarse.method == 0 ? gauss_radau_right(coarse.k + 1) : gauss_lobatto(coarse.k + 1);
  const int ncc = coarse.nt_cell;
  Mat P(fine.n_t, coarse.n_t);
  for (int m = 0; m < fine.c; ++m)
    for (int j = 0; j < fine.nt_cell; ++j) {
      const int i = m * fine.nt_cell + j;
      const double t = (m + fpos[j]) * fine.tau;          // time from the slab start
      const double sc = t / coarse.tau;
      int M = (int)std::ceil(sc - 1e-12) - 1;              // coarse cell (t_{M}, t_{M+1}]
      M = std::min(std::max(M, 0), coarse.c - 1);
      Mat V, D;
      lagrange(cnodes, Vec{sc - M}, V, D);
      if (coarse.method == 0) {
        for (int b = 0; b < ncc; ++b) P(i, M * ncc + b) = V(0, b);
      } else {
        for (int b = 0; b < ncc; ++b) P(i, M * ncc + b) = V(0, b + 1);
        if (M > 0) P(i, M * ncc - 1) += V(0, 0);
      }
    }
  return P;
}

}  // namespace hm
}  // namespace stmg
