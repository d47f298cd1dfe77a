// FP64 flexible GMRES(m) preconditioned by one space-time multigrid V-cycle per
// iteration (Section 4: GMRES with one V-cycle per iteration).  Right
// preconditioning; classical Gram-Schmidt applied twice (two fused multi-dot /
// multi-axpy passes per Arnoldi step); Givens rotations and the small least-
// squares problem on the host.  The residual, the Krylov basis and the solution
// update are FP64; with precision FP32 the V-cycle (operator, smoother,
// transfers, coarse solve) runs in FP32 on a cast of the Arnoldi vector, and the
// flexible basis Z is kept in FP32.  Convergence is judged on the true FP64
// residual at every restart and at exit.
#include <chrono>
#include <cmath>

#include "handle.hpp"

namespace stmg {

stmg_status cnn_precondition(stmg_handle* h, const double* v, double* z, double* tmp, bool* used);

namespace {

void ensure_workspace(stmg_handle* h, long long n, int m) {
  bool need32 = h->cfg.precision != STMG_PREC_FP64;
  if (h->krylov_m == m && h->V.get()) return;
  h->V.alloc(sizeof(double) * n * (m + 1));
  h->w.alloc(sizeof(double) * n);
  h->red.alloc(sizeof(double) * RED_BLOCKS * PS);
  h->dots.alloc(sizeof(double) * (2 * m + 6));   // dot products and norms, then squared basis scales
  if (need32) {
    h->Z32.alloc(sizeof(float) * n * m);
    h->tmp32a.alloc(sizeof(float) * n);
    if (h->cfg.precision == STMG_PREC_LEARNED) h->tmp32b.alloc(sizeof(float) * n);
    h->Z64.alloc(sizeof(double) * n);   // one FP64 scratch vector (cast of z_j)
  } else {
    h->Z64.alloc(sizeof(double) * n * m);
  }
  h->krylov_m = m;
}

}  // namespace

// ||v - w||_2 with w = S z already computed; tmp is overwritten
static double stage_residual(stmg_handle* h, const double* v, const double* w, double* tmp, long long n) {
  hipStream_t s = h->stream;
  copy<double>(w, tmp, n, s);
  axpby<double>(1.0, v, -1.0, tmp, n, s);
  norm2_check<double>(tmp, n, h->dots.as<double>(), h->red.as<double>(), s);
  std::vector<double> r = download<double>(h->dots.get(), 2, s);
  return r[1] != 0.0 ? INFINITY : std::sqrt(r[0]);
}

stmg_status fgmres(stmg_handle* h, const double* b_in, double* x, stmg_solve_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = h->stream;
  Level& L = *h->levels[0];
  const int n_t = h->tm.n_t;
  const long long n = L.nst(n_t);
  const int m = h->cfg.restart;
  const bool mixed = h->cfg.precision != STMG_PREC_FP64;
  const bool learned = h->cfg.precision == STMG_PREC_LEARNED;
  if (learned && !h->cnn) fail(STMG_E_STATE, "precision LEARNED needs a network (stmg_cnn_create)");
  ensure_workspace(h, n, m);
  double* V = h->V.as<double>();
  double* b = h->w.as<double>();
  double* dots = h->dots.as<double>();
  double* red = h->red.as<double>();
  double* s2d = dots + m + 4;
  stmg_solve_info inf{};
  h->timer.on = true;
  h->timer.reset();
  h->ktimer.on = true;
  h->timer.mark(TB_OTHER, s);
  // homogeneous Dirichlet data: zero b and x on the boundary
  copy<double>(b_in, b, n, s);
  boundary_axpby<double>(L.bidx.as<int>(), L.nb, L.g.nx, n_t, 0.0, b, 0.0, b, s);
  boundary_axpby<double>(L.bidx.as<int>(), L.nb, L.g.nx, n_t, 0.0, x, 0.0, x, s);
  norm2_check<double>(b, n, dots, red, s);
  std::vector<double> nb2 = download<double>(dots, 2, s);
  if (nb2[1] != 0.0) { h->timer.on = false; h->ktimer.on = false; fail(STMG_E_NONFINITE, "right-hand side contains NaN or Inf"); }
  norm2_check<double>(x, n, dots, red, s);
  std::vector<double> nx2 = download<double>(dots, 2, s);
  if (nx2[1] != 0.0) { h->timer.on = false; h->ktimer.on = false; fail(STMG_E_NONFINITE, "initial guess contains NaN or Inf"); }
  const double bnorm = std::sqrt(nb2[0]);
  stmg_status status = STMG_OK;
  int it = 0;
  double rel = 0.0;
  // the learned stage is no longer evaluated in this solve after CNN_MAX_REJECT rejections in a row
  constexpr int CNN_MAX_REJECT = 3;
  constexpr double GS_REFINE = 0.125;
  int cnn_reject_run = 0;
  double rho_plain = -1.0;     // ||v - S V(v)|| / ||v|| of the last plain preconditioner application
  if (bnorm == 0.0) {
    fill<double>(x, 0.0, n, s);
  } else {
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    // Basis vectors are stored unnormalised, v_i = sc[i] V_i, and the scales enter the Gram-Schmidt
    // coefficients (device copy s2d = sc^2), the Hessenberg entries and the update of x, which saves
    // a scaling pass over every new vector.  A V-cycle is linear, so Z_i = V(V_i) = V(v_i) / sc[i].
    // The learned stage is not linear and sees unit vectors (sc = 1, explicit scaling).
    const bool lazy = !learned;
    std::vector<double> sc(m + 1, 1.0), s2h(m + 1, 1.0);
    auto set_scale = [&](int i, double v) {
      sc[i] = v;
      s2h[i] = v * v;
      STMG_HIP(hipMemcpyAsync(s2d + i, &s2h[i], sizeof(double), hipMemcpyHostToDevice, s));
    };
    for (;;) {
      // true residual r = b - S x into V_0
      h->timer.mark(TB_OP, s);
      vmult<double>(h, 0, x, V);
      h->timer.mark(TB_OTHER, s);
      axpby<double>(1.0, b, -1.0, V, n, s);
      norm2_check<double>(V, n, dots, red, s);
      std::vector<double> r2 = download<double>(dots, 2, s);
      if (r2[1] != 0.0) { status = STMG_E_NONFINITE; break; }
      double beta = std::sqrt(r2[0]);
      rel = beta / bnorm;
      if (rel <= h->cfg.rtol) break;
      if (it >= h->cfg.max_iter) { status = STMG_E_NOCONV; break; }
      if (it > 0) inf.restarts++;
      if (lazy) set_scale(0, 1.0 / beta);
      else scal<double>(1.0 / beta, V, n, s);
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = beta;
      int jused = 0;
      bool bad = false;
      for (int j = 0; j < m; ++j) {
        double* vj = V + (size_t)j * n;
        double* vn = V + (size_t)(j + 1) * n;
        double* zj;   // FP64 view of z_j for the operator
        // z_j = Prec(v_j)
        h->timer.mark(TB_GMG, s);
        if (mixed) {
          float* z32 = h->Z32.as<float>() + (size_t)j * n;
          double* z64 = h->Z64.as<double>();
          const bool judge = learned && cnn_reject_run < CNN_MAX_REJECT;
          bool used = false;
          if (judge && rho_plain >= 0.0) {
            cnn_precondition(h, vj, z64, vn, &used);
            cast_d2f(z64, z32, n, s);
          } else {
            cast_d2f(vj, h->tmp32a.as<float>(), n, s);
            vcycle<float>(h, 0, h->tmp32a.as<float>(), z32);
          }
          cast_f2d(z32, z64, n, s);
          zj = z64;
          h->timer.mark(TB_OP, s);
          vmult<double>(h, 0, zj, vn);
          if (judge) {
            // plain STMG judges the stage: accept it only if ||v_j - S z_j|| does not exceed
            // what the last plain V-cycle reached (||v_j|| = 1); otherwise redo z_j = V(v_j)
            h->timer.mark(TB_OTHER, s);
            double rho = stage_residual(h, vj, vn, z64, n);
            if (used && !(rho <= rho_plain)) {
              used = false;
              h->timer.mark(TB_GMG, s);
              cast_d2f(vj, h->tmp32a.as<float>(), n, s);
              vcycle<float>(h, 0, h->tmp32a.as<float>(), z32);
              cast_f2d(z32, z64, n, s);
              h->timer.mark(TB_OP, s);
              vmult<double>(h, 0, z64, vn);
              h->timer.mark(TB_OTHER, s);
              rho = stage_residual(h, vj, vn, z64, n);
              cnn_reject_run++;
            } else if (used) {
              cnn_reject_run = 0;
            } else if (rho_plain >= 0.0) {
              cnn_reject_run++;        // rejected by the network's own residual test
            }
            if (!used) rho_plain = rho;
          }
          if (learned) { if (used) inf.cnn_used++; else inf.cnn_fallbacks++; }
        } else {
          zj = h->Z64.as<double>() + (size_t)j * n;
          vcycle<double>(h, 0, vj, zj);
          // w = S z_j
          h->timer.mark(TB_OP, s);
          vmult<double>(h, 0, zj, vn);
        }
        h->timer.mark(TB_OTHER, s);
        // classical Gram-Schmidt: one pass reads V once for V^T w and ||w||^2, one fused pass
        // updates w and returns ||w'||^2; a second pass follows when the pass cancelled most of
        // w (||w'|| < GS_REFINE ||w||) or when two passes are requested
        std::vector<double> hc(j + 1, 0.0);
        std::vector<double> w2;
        for (int pass = 0; pass < 2; ++pass) {
          // dots[0..j] = V^T w, dots[j+1] = ||w||^2, then dots[j+2..j+3] = ||w'||^2 and the
          // non-finite flag of the update: one read-back per pass
          multi_dot(V, n, j + 1, vn, n, dots, red, s, true);
          multi_axpy_neg_norm(V, n, j + 1, dots, vn, n, dots + j + 2, red, s, lazy ? s2d : nullptr);
          std::vector<double> hv = download<double>(dots, j + 4, s);
          w2.assign(hv.begin() + j + 2, hv.begin() + j + 4);
          for (int i = 0; i <= j; ++i) hc[i] += hv[i] * sc[i] * sc[j];
          const double ww = hv[j + 1];
          if (!std::isfinite(ww) || w2[1] != 0.0) { bad = true; break; }
          if (h->cfg.gram_schmidt == 0 && w2[0] >= GS_REFINE * GS_REFINE * ww) break;
        }
        if (bad) break;
        const double hraw = std::sqrt(w2[0]), hn = sc[j] * hraw;
        for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hc[i];
        H[(size_t)(j + 1) * m + j] = hn;
        if (hraw > 0.0) {
          if (lazy) set_scale(j + 1, 1.0 / hraw);
          else scal<double>(1.0 / hraw, vn, n, s);
        }
        for (int i = 0; i < j; ++i) {
          double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
          H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
          H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
        }
        double a = H[(size_t)j * m + j], c = H[(size_t)(j + 1) * m + j];
        double den = std::hypot(a, c);
        cs[j] = den > 0 ? a / den : 1.0;
        sn[j] = den > 0 ? c / den : 0.0;
        H[(size_t)j * m + j] = den;
        H[(size_t)(j + 1) * m + j] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        ++it;
        jused = j + 1;
        if (std::fabs(g[j + 1]) / bnorm <= h->cfg.rtol || it >= h->cfg.max_iter || hn == 0.0) break;
      }
      if (bad) { status = STMG_E_NONFINITE; break; }
      // y = R^{-1} g ; x += Z y
      for (int i = jused - 1; i >= 0; --i) {
        double sum = g[i];
        for (int k = i + 1; k < jused; ++k) sum -= H[(size_t)i * m + k] * y[k];
        y[i] = sum / H[(size_t)i * m + i];
      }
      for (int i = 0; i < jused; ++i) y[i] *= sc[i];
      STMG_HIP(hipMemcpyAsync(dots, y.data(), sizeof(double) * jused, hipMemcpyHostToDevice, s));
      if (mixed) multi_axpy_acc<float>(h->Z32.as<float>(), n, jused, dots, x, n, s);
      else multi_axpy_acc<double>(h->Z64.as<double>(), n, jused, dots, x, n, s);
      STMG_HIP(hipStreamSynchronize(s));
    }
  }
  h->timer.mark(TB_OTHER, s);
  STMG_HIP(hipStreamSynchronize(s));
  double buckets[4] = {0, 0, 0, 0};
  h->timer.accumulate(buckets);
  h->timer.on = false;
  h->ktimer.flush();
  h->ktimer.on = false;
  inf.iterations = it;
  inf.rel_residual = rel;
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  inf.t_smoother = buckets[TB_SMOOTH];
  inf.t_gmg_other = buckets[TB_GMG];
  inf.t_operator = buckets[TB_OP];
  inf.t_other = buckets[TB_OTHER];
  if (info) *info = inf;
  return status;
}

}  // namespace stmg
