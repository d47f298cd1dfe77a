// C ABI entry points of libstmg (declared in include/stmg.h).  Every entry
// point validates its arguments, runs the C++ implementation and converts any
// exception into an stmg_status plus a thread-local message.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "handle.hpp"

namespace {

thread_local std::string g_last_error;

template <class F>
stmg_status guarded(F&& f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const stmg::Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return STMG_E_NOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return STMG_E_HIP;
  } catch (...) {
    g_last_error = "unknown error";
    return STMG_E_HIP;
  }
}

void check_config(const stmg_config* c) {
  using stmg::fail;
  if (!c) fail(STMG_E_ARG, "cfg is NULL");
  if (c->abi_version != STMG_ABI_VERSION) fail(STMG_E_ARG, "abi_version mismatch");
  if (c->dim != 2 && c->dim != 3) fail(STMG_E_ARG, "dim must be 2 or 3");
  if (c->problem != STMG_HEAT && c->problem != STMG_WAVE) fail(STMG_E_ARG, "problem must be heat (0) or wave (1)");
  if (c->time_method != STMG_DG && c->time_method != STMG_CGP) fail(STMG_E_ARG, "time_method must be dG (0) or cGP (1)");
  if (c->p < 1 || c->p > 4) fail(STMG_E_UNSUPPORTED, "p must be in 1..4");
  if (c->time_method == STMG_DG && (c->k < 0 || c->k > 5)) fail(STMG_E_UNSUPPORTED, "dG degree k must be in 0..5");
  if (c->time_method == STMG_CGP && (c->k < 1 || c->k > 5)) fail(STMG_E_UNSUPPORTED, "cGP degree k must be in 1..5");
  if (c->n_time_cells < 1) fail(STMG_E_ARG, "n_time_cells must be >= 1");
  for (int d = 0; d < c->dim; ++d)
    if (c->n_cells[d] < 1) fail(STMG_E_ARG, "n_cells must be >= 1");
  if (!(c->tau > 0.0) || !std::isfinite(c->tau)) fail(STMG_E_ARG, "tau must be positive");
  for (int d = 0; d < c->dim; ++d)
    if (!(c->hi[d] > c->lo[d])) fail(STMG_E_ARG, "hi must exceed lo");
  if (c->n_smooth < 1) fail(STMG_E_ARG, "n_smooth must be >= 1");
  if (c->min_p < 1) fail(STMG_E_ARG, "min_p must be >= 1");
  if (c->coarse_cells < 1) fail(STMG_E_ARG, "coarse_cells must be >= 1");
  if (c->precision < 0 || c->precision > 2) fail(STMG_E_ARG, "precision must be 0, 1 or 2");
  if (c->restart < 1 || c->restart > 200) fail(STMG_E_ARG, "restart must be in 1..200");
  if (c->gram_schmidt != 0 && c->gram_schmidt != 1) fail(STMG_E_ARG, "gram_schmidt must be 0 or 1");
  if (c->asm_variant < 0 || c->asm_variant > 2) fail(STMG_E_ARG, "asm_variant must be 0, 1 or 2");
  if (c->time_mg != 0 && c->time_mg != 1) fail(STMG_E_ARG, "time_mg must be 0 or 1");
  if (c->kernel_path < STMG_PATH_DEFAULT || c->kernel_path > STMG_PATH_COLOUR)
    fail(STMG_E_ARG, "kernel_path must be 0, 1 or 2");
  if (c->max_iter < 1) fail(STMG_E_ARG, "max_iter must be >= 1");
  if (!(c->rtol > 0.0)) fail(STMG_E_ARG, "rtol must be positive");
  if (c->vcycle_dtypes < 0 || c->vcycle_dtypes > 3) fail(STMG_E_ARG, "vcycle_dtypes must be in 0..3");
  long long nx = 1;
  for (int d = 0; d < c->dim; ++d) nx *= (long long)c->p * c->n_cells[d] + 1;
  int per = c->time_method == STMG_DG ? c->k + 1 : c->k;
  long long nst = nx * per * c->n_time_cells;
  if (nst >= (1LL << 31)) fail(STMG_E_UNSUPPORTED, "more than 2^31 space-time DoFs");
}

// the temporal parameters the library supports (the same limits as stmg_create)
void check_temporal(int problem, int method, int k, int c, double tau) {
  using stmg::fail;
  if (problem != STMG_HEAT && problem != STMG_WAVE) fail(STMG_E_ARG, "problem must be heat (0) or wave (1)");
  if (method != STMG_DG && method != STMG_CGP) fail(STMG_E_ARG, "method must be dG (0) or cGP (1)");
  if (method == STMG_DG && (k < 0 || k > 5)) fail(STMG_E_UNSUPPORTED, "dG degree k must be in 0..5");
  if (method == STMG_CGP && (k < 1 || k > 5)) fail(STMG_E_UNSUPPORTED, "cGP degree k must be in 1..5");
  if (c < 1 || c > 4096) fail(STMG_E_ARG, "the number of time cells must be in 1..4096");
  if (!(tau > 0.0) || !std::isfinite(tau)) fail(STMG_E_ARG, "tau must be positive");
}

// every multilinear cell must have a positive Jacobian determinant at its corners
void check_vertices(const stmg_config* c, const double* v) {
  int d = c->dim;
  int nx = c->n_cells[0], ny = c->n_cells[1], nz = d == 3 ? c->n_cells[2] : 1;
  auto P = [&](int x, int y, int z, int k) {
    return v[(((size_t)z * (ny + 1) + y) * (nx + 1) + x) * d + k];
  };
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x)
        for (int corner = 0; corner < (1 << d); ++corner) {
          int bx = corner & 1, by = (corner >> 1) & 1, bz = (corner >> 2) & 1;
          int sx = bx ? -1 : 1, sy = by ? -1 : 1, sz = bz ? -1 : 1;
          double e[3][3];
          for (int k = 0; k < d; ++k) {
            e[0][k] = sx * (P(x + 1 - bx, y + by, z + bz, k) - P(x + bx, y + by, z + bz, k));
            e[1][k] = sy * (P(x + bx, y + 1 - by, z + bz, k) - P(x + bx, y + by, z + bz, k));
            if (d == 3) e[2][k] = sz * (P(x + bx, y + by, z + 1 - bz, k) - P(x + bx, y + by, z + bz, k));
          }
          double det;
          if (d == 2) det = e[0][0] * e[1][1] - e[0][1] * e[1][0];
          else
            det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                  e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                  e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
          if (!(det > 0.0)) stmg::fail(STMG_E_ARG, "inverted or degenerate cell in the vertex lattice");
        }
}

stmg::Level& level_of(stmg_handle* h, int level) {
  if (!h) stmg::fail(STMG_E_ARG, "handle is NULL");
  if (level < 0 || level >= (int)h->levels.size()) stmg::fail(STMG_E_ARG, "level out of range");
  return *h->levels[level];
}

void check_dtype(stmg_handle* h, int dtype, bool need_vcycle_data, int level) {
  if (dtype != STMG_F64 && dtype != STMG_F32) stmg::fail(STMG_E_ARG, "dtype must be 0 (f64) or 1 (f32)");
  if (!need_vcycle_data) return;
  stmg::Level& L = *h->levels[level];
  if (dtype == STMG_F64 && !L.has64) stmg::fail(STMG_E_STATE, "FP64 V-cycle data not built (vcycle_dtypes)");
  if (dtype == STMG_F32 && !L.has32) stmg::fail(STMG_E_STATE, "FP32 V-cycle data not built (vcycle_dtypes)");
}

}  // namespace

stmg_handle::~stmg_handle() {
  if (stream) (void)hipStreamSynchronize(stream);
  else (void)hipDeviceSynchronize();
  stmg::cnn_free(cnn);
}

extern "C" {

stmg_status stmg_create(const stmg_config* cfg, const double* vertices, const double* coeff, void* hip_stream,
                        stmg_handle** out) {
  return guarded([&]() -> stmg_status {
    if (!out) stmg::fail(STMG_E_ARG, "out is NULL");
    check_config(cfg);
    if (vertices) check_vertices(cfg, vertices);
    if (vertices && cfg->asm_variant == 1)
      stmg::fail(STMG_E_UNSUPPORTED, "the separable smoother (asm_variant 1) needs a Cartesian mesh");
    if (vertices && cfg->asm_variant == 2)
      stmg::fail(STMG_E_UNSUPPORTED, "the vertex-patch smoother (asm_variant 2) needs a Cartesian mesh");
    auto t0 = std::chrono::steady_clock::now();
    int64_t bytes0 = stmg::DevBuf::total_bytes();
    std::unique_ptr<stmg_handle> h(new stmg_handle());
    h->cfg = *cfg;
    h->stream = static_cast<hipStream_t>(hip_stream);
    STMG_HIP(hipGetDevice(&h->device));
    stmg::noalloc_init(h->device);
    int dt = cfg->vcycle_dtypes;
    if (dt == 0) dt = cfg->precision == STMG_PREC_FP64 ? 1 : 2;
    h->want64 = (dt & 1) != 0;
    h->want32 = (dt & 2) != 0;
    stmg::build_hierarchy(h.get(), vertices, coeff);
    h->setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    h->bytes_at_create = stmg::DevBuf::total_bytes() - bytes0;
    *out = h.release();
    return STMG_OK;
  });
}

stmg_status stmg_vmult(stmg_handle* h, int level, int dtype, const void* x, void* y) {
  return guarded([&]() -> stmg_status {
    level_of(h, level);
    check_dtype(h, dtype, false, level);
    if (!x || !y) stmg::fail(STMG_E_ARG, "x or y is NULL");
    if (x == y) stmg::fail(STMG_E_ARG, "x and y must not alias");
    if (dtype == STMG_F64) stmg::vmult<double>(h, level, (const double*)x, (double*)y);
    else stmg::vmult<float>(h, level, (const float*)x, (float*)y);
    return STMG_OK;
  });
}

stmg_status stmg_vmult_noalloc(stmg_handle* h, int level, int dtype, const void* x, void* y) {
  return guarded([&]() -> stmg_status {
    level_of(h, level);
    check_dtype(h, dtype, false, level);
    if (!x || !y) stmg::fail(STMG_E_ARG, "x or y is NULL");
    if (x == y) stmg::fail(STMG_E_ARG, "x and y must not alias");
    if (dtype == STMG_F64) stmg::vmult_noalloc<double>(h, level, (const double*)x, (double*)y);
    else stmg::vmult_noalloc<float>(h, level, (const float*)x, (float*)y);
    return STMG_OK;
  });
}

stmg_status stmg_smooth(stmg_handle* h, int level, int dtype, const void* b, void* x, int n_steps) {
  return guarded([&]() -> stmg_status {
    level_of(h, level);
    if (level == (int)h->levels.size() - 1) stmg::fail(STMG_E_ARG, "the coarsest level has no smoother");
    check_dtype(h, dtype, true, level);
    if (!b || !x) stmg::fail(STMG_E_ARG, "b or x is NULL");
    if (n_steps < 0) stmg::fail(STMG_E_ARG, "n_steps must be >= 0");
    if (dtype == STMG_F64) stmg::smooth<double>(h, level, (const double*)b, (double*)x, n_steps);
    else stmg::smooth<float>(h, level, (const float*)b, (float*)x, n_steps);
    return STMG_OK;
  });
}

stmg_status stmg_vcycle(stmg_handle* h, int dtype, const void* r, void* z) {
  return guarded([&]() -> stmg_status {
    level_of(h, 0);
    check_dtype(h, dtype, true, 0);
    if (!r || !z) stmg::fail(STMG_E_ARG, "r or z is NULL");
    if (r == z) stmg::fail(STMG_E_ARG, "r and z must not alias");
    if (dtype == STMG_F64) stmg::vcycle<double>(h, 0, (const double*)r, (double*)z);
    else stmg::vcycle<float>(h, 0, (const float*)r, (float*)z);
    return STMG_OK;
  });
}

stmg_status stmg_mg_step(stmg_handle* h, int dtype, const void* b, void* x, void* r, void* z) {
  return guarded([&]() -> stmg_status {
    level_of(h, 0);
    check_dtype(h, dtype, true, 0);
    if (!b || !x || !r || !z) stmg::fail(STMG_E_ARG, "b, x, r or z is NULL");
    const void* v[4] = {b, x, r, z};
    for (int i = 0; i < 4; ++i)
      for (int j = i + 1; j < 4; ++j)
        if (v[i] == v[j]) stmg::fail(STMG_E_ARG, "b, x, r and z must not alias");
    if (dtype == STMG_F64) stmg::mg_step<double>(h, (const double*)b, (double*)x, (double*)r, (double*)z);
    else stmg::mg_step<float>(h, (const float*)b, (float*)x, (float*)r, (float*)z);
    return STMG_OK;
  });
}

stmg_status stmg_prolongate(stmg_handle* h, int level, int dtype, const void* coarse, void* fine) {
  return guarded([&]() -> stmg_status {
    level_of(h, level);
    if (level + 1 >= (int)h->levels.size()) stmg::fail(STMG_E_ARG, "level has no coarser level");
    check_dtype(h, dtype, true, level);
    if (!coarse || !fine) stmg::fail(STMG_E_ARG, "NULL vector");
    if (dtype == STMG_F64) stmg::prolongate<double>(h, level, (const double*)coarse, (double*)fine, false);
    else stmg::prolongate<float>(h, level, (const float*)coarse, (float*)fine, false);
    return STMG_OK;
  });
}

stmg_status stmg_restrict(stmg_handle* h, int level, int dtype, const void* fine, void* coarse) {
  return guarded([&]() -> stmg_status {
    level_of(h, level);
    if (level + 1 >= (int)h->levels.size()) stmg::fail(STMG_E_ARG, "level has no coarser level");
    check_dtype(h, dtype, true, level);
    if (!coarse || !fine) stmg::fail(STMG_E_ARG, "NULL vector");
    if (dtype == STMG_F64) stmg::restrict_<double>(h, level, (const double*)fine, (double*)coarse);
    else stmg::restrict_<float>(h, level, (const float*)fine, (float*)coarse);
    return STMG_OK;
  });
}

stmg_status stmg_solve(stmg_handle* h, const double* b, double* x, stmg_solve_info* info) {
  return guarded([&]() -> stmg_status {
    level_of(h, 0);
    if (!b || !x) stmg::fail(STMG_E_ARG, "b or x is NULL");
    if ((const void*)b == (const void*)x) stmg::fail(STMG_E_ARG, "b and x must not alias");
    check_dtype(h, h->cfg.precision == STMG_PREC_FP64 ? STMG_F64 : STMG_F32, true, 0);
    stmg_status st = stmg::fgmres(h, b, x, info);
    if (st == STMG_E_NOCONV) g_last_error = "FGMRES did not reach rtol within max_iter";
    if (st == STMG_E_NONFINITE) g_last_error = "non-finite value in the iteration";
    return st;
  });
}

stmg_status stmg_kernel_stats_get(stmg_handle* h, stmg_kernel_stats* out, int reset) {
  return guarded([&]() -> stmg_status {
    level_of(h, 0);
    if (!out) stmg::fail(STMG_E_ARG, "out is NULL");
    h->ktimer.flush();
    out->n_operator = h->ktimer.n[0];
    out->n_smoother = h->ktimer.n[1];
    out->t_operator = h->ktimer.t[0];
    out->t_smoother = h->ktimer.t[1];
    if (reset) {
      h->ktimer.n[0] = h->ktimer.n[1] = 0;
      h->ktimer.t[0] = h->ktimer.t[1] = 0.0;
    }
    return STMG_OK;
  });
}

stmg_status stmg_set_precision(stmg_handle* h, int precision) {
  return guarded([&]() -> stmg_status {
    level_of(h, 0);
    if (precision < 0 || precision > 2) stmg::fail(STMG_E_ARG, "precision must be 0, 1 or 2");
    check_dtype(h, precision == STMG_PREC_FP64 ? STMG_F64 : STMG_F32, true, 0);
    if (precision != h->cfg.precision) {
      h->cfg.precision = precision;
      h->krylov_m = 0;      // workspace layout depends on the precision
    }
    return STMG_OK;
  });
}

stmg_status stmg_cnn_create(stmg_handle* h, int n_layers, const int32_t* channels) {
  return guarded([&]() -> stmg_status {
    level_of(h, 0);
    if (!channels) stmg::fail(STMG_E_ARG, "channels is NULL");
    if (n_layers < 1 || n_layers > 6) stmg::fail(STMG_E_ARG, "n_layers must be in 1..6");
    std::vector<int> ch(channels, channels + n_layers + 1);
    stmg::cnn_create(h, n_layers, ch.data());
    h->krylov_m = 0;
    return STMG_OK;
  });
}

stmg_status stmg_cnn_param_count(stmg_handle* h, int64_t* n) {
  return guarded([&]() -> stmg_status {
    level_of(h, 0);
    if (!n) stmg::fail(STMG_E_ARG, "n is NULL");
    *n = stmg::cnn_param_count(h);
    return STMG_OK;
  });
}

stmg_status stmg_cnn_set_params(stmg_handle* h, const float* params, int64_t n) {
  return guarded([&]() -> stmg_status {
    level_of(h, 0);
    if (!params) stmg::fail(STMG_E_ARG, "params is NULL");
    stmg::cnn_set_params(h, params, n);
    return STMG_OK;
  });
}

stmg_status stmg_cnn_get_params(stmg_handle* h, float* params, int64_t n) {
  return guarded([&]() -> stmg_status {
    level_of(h, 0);
    if (!params) stmg::fail(STMG_E_ARG, "params is NULL");
    stmg::cnn_get_params(h, params, n);
    return STMG_OK;
  });
}

stmg_status stmg_slab_rhs(stmg_handle* h, const double* F, const double* F0, const double* u0, const double* v0,
                          double* b) {
  return guarded([&]() -> stmg_status {
    level_of(h, 0);
    if (!b) stmg::fail(STMG_E_ARG, "b is NULL");
    if ((const void*)b == (const void*)F) stmg::fail(STMG_E_ARG, "b must not alias F");
    stmg::slab_rhs(h, F, F0, u0, v0, b);
    return STMG_OK;
  });
}

stmg_status stmg_node_coordinates(stmg_handle* h, double* xyz) {
  return guarded([&]() -> stmg_status {
    level_of(h, 0);
    if (!xyz) stmg::fail(STMG_E_ARG, "xyz is NULL");
    stmg::node_coordinates(h, xyz);
    return STMG_OK;
  });
}

stmg_status stmg_point_values(stmg_handle* h, const double* U, int n_planes, int npts, const double* pts,
                              double* out) {
  return guarded([&]() -> stmg_status {
    level_of(h, 0);
    if (!U || !pts || !out) stmg::fail(STMG_E_ARG, "NULL argument");
    if (n_planes < 1 || n_planes > h->tm.n_t) stmg::fail(STMG_E_ARG, "n_planes must be in 1..n_t");
    if (npts < 0) stmg::fail(STMG_E_ARG, "npts must be >= 0");
    if (npts > 0) stmg::point_values(h, U, n_planes, npts, pts, out);
    return STMG_OK;
  });
}

stmg_status stmg_wave_velocity(stmg_handle* h, const double* U, const double* u0, const double* v0, double* V) {
  return guarded([&]() -> stmg_status {
    level_of(h, 0);
    if (h->cfg.problem != STMG_WAVE) stmg::fail(STMG_E_UNSUPPORTED, "velocity recovery needs the wave problem");
    if (!U || !V || (const void*)U == (const void*)V) stmg::fail(STMG_E_ARG, "bad U / V");
    stmg::wave_velocity(h, U, u0, v0, V);
    return STMG_OK;
  });
}

stmg_status stmg_cnn_forward(stmg_handle* h, const double* r, double* z) {
  return guarded([&]() -> stmg_status {
    level_of(h, 0);
    if (!r || !z || (const void*)r == (const void*)z) stmg::fail(STMG_E_ARG, "bad r / z");
    stmg::cnn_forward(h, r, z);
    STMG_HIP(hipStreamSynchronize(h->stream));
    return STMG_OK;
  });
}

stmg_status stmg_cnn_param_grad(stmg_handle* h, const double* r, const double* dz, float* grad, int64_t n) {
  return guarded([&]() -> stmg_status {
    level_of(h, 0);
    if (!r || !dz || !grad) stmg::fail(STMG_E_ARG, "NULL argument");
    if (n != stmg::cnn_param_count(h)) stmg::fail(STMG_E_ARG, "parameter count mismatch");
    stmg::cnn_param_grad(h, r, dz, grad);
    return STMG_OK;
  });
}

stmg_status stmg_cnn_train_step(stmg_handle* h, const double* r, const double* e, double lr, double* loss) {
  return guarded([&]() -> stmg_status {
    level_of(h, 0);
    if (!r || !e) stmg::fail(STMG_E_ARG, "NULL argument");
    if (!(lr > 0.0)) stmg::fail(STMG_E_ARG, "lr must be positive");
    double l = stmg::cnn_train_step(h, r, e, lr);
    if (loss) *loss = l;
    return STMG_OK;
  });
}

stmg_status stmg_set_omega(stmg_handle* h, int level, double omega) {
  return guarded([&]() -> stmg_status {
    stmg::Level& L = level_of(h, level);
    if (!(omega > 0.0) || !std::isfinite(omega)) stmg::fail(STMG_E_ARG, "omega must be positive");
    L.omega = omega;
    return STMG_OK;
  });
}

stmg_status stmg_query(stmg_handle* h, stmg_info* info) {
  return guarded([&]() -> stmg_status {
    level_of(h, 0);
    if (!info) stmg::fail(STMG_E_ARG, "info is NULL");
    *info = stmg_info{};
    info->n_levels = (int)h->levels.size();
    info->n_t = h->tm.n_t;
    info->nt_cell = h->tm.nt_cell;
    int nnz = 0;
    for (const stmg::hm::Mat* A : {&h->tm.M_T, &h->tm.N_T})
      for (int i = 0; i < A->r; ++i)
        for (int j = 0; j < A->c; ++j) nnz += ((*A)(i, j) != 0.0);
    info->temporal_nnz = nnz;
    for (size_t l = 0; l < h->levels.size(); ++l) {
      const stmg::Level& L = *h->levels[l];
      info->n_x[l] = L.g.nx;
      info->p[l] = L.p;
      for (int d = 0; d < 3; ++d) info->cells[l][d] = L.cells[d];
      info->omega[l] = L.omega;
      info->n_t_level[l] = L.n_t();
      info->nt_cell_level[l] = L.ts->tm.nt_cell;
    }
    info->coarse_unknowns = h->levels.back()->cm;
    info->device_bytes = h->bytes_at_create;
    info->eig_resolves = h->eig_resolves;
    info->setup_seconds = h->setup_seconds;
    return STMG_OK;
  });
}

void stmg_destroy(stmg_handle* h) {
  try {
    delete h;
  } catch (...) {
  }
}

stmg_status stmg_temporal_matrices(int problem, int method, int k, int n_time_cells, double tau, int64_t cap,
                                   int32_t* n_t, double* M_T, double* A_T, double* N_T) {
  return guarded([&] {
    check_temporal(problem, method, k, n_time_cells, tau);
    if (!n_t) stmg::fail(STMG_E_ARG, "n_t is NULL");
    const stmg::hm::Temporal T = stmg::hm::temporal(problem, method, k, n_time_cells, tau);
    *n_t = T.n_t;
    const stmg::hm::Mat* src[3] = {&T.M_T, &T.A_T, &T.N_T};
    double* dst[3] = {M_T, A_T, N_T};
    for (int m = 0; m < 3; ++m) {
      if (!dst[m]) continue;
      if (cap < (int64_t)T.n_t * T.n_t) stmg::fail(STMG_E_ARG, "cap is smaller than n_t * n_t");
      std::copy(src[m]->a.begin(), src[m]->a.end(), dst[m]);
    }
    return STMG_OK;
  });
}

stmg_status stmg_temporal_cell_factors(int problem, int method, int k, double tau, int64_t cap, int32_t* nt_cell,
                                       double* M_tau, double* N_tilde) {
  return guarded([&] {
    check_temporal(problem, method, k, 1, tau);
    if (!nt_cell) stmg::fail(STMG_E_ARG, "nt_cell is NULL");
    const stmg::hm::Temporal T = stmg::hm::temporal(problem, method, k, 1, tau);
    *nt_cell = T.nt_cell;
    const stmg::hm::Mat* src[2] = {&T.M_tau, &T.N_tilde};
    double* dst[2] = {M_tau, N_tilde};
    for (int m = 0; m < 2; ++m) {
      if (!dst[m]) continue;
      if (cap < (int64_t)T.nt_cell * T.nt_cell) stmg::fail(STMG_E_ARG, "cap is smaller than nt_cell * nt_cell");
      std::copy(src[m]->a.begin(), src[m]->a.end(), dst[m]);
    }
    return STMG_OK;
  });
}

stmg_status stmg_temporal_dof_times(int problem, int method, int k, int n_time_cells, double tau, double t0,
                                    int64_t cap, int32_t* n_t, double* times) {
  return guarded([&] {
    check_temporal(problem, method, k, n_time_cells, tau);
    if (!n_t) stmg::fail(STMG_E_ARG, "n_t is NULL");
    if (!std::isfinite(t0)) stmg::fail(STMG_E_ARG, "t0 must be finite");
    const stmg::hm::Temporal T = stmg::hm::temporal(problem, method, k, n_time_cells, tau);
    *n_t = T.n_t;
    if (times) {
      if (cap < (int64_t)T.n_t) stmg::fail(STMG_E_ARG, "cap is smaller than n_t");
      const stmg::hm::Vec pos = stmg::hm::dof_positions(T);
      for (int m = 0; m < n_time_cells; ++m)
        for (int l = 0; l < T.nt_cell; ++l) times[m * T.nt_cell + l] = t0 + (m + pos[l]) * tau;
    }
    return STMG_OK;
  });
}

stmg_status stmg_transfer_1d(int p_coarse, int n_coarse, int p_fine, int n_fine, int64_t cap, int32_t* rows,
                             int32_t* cols, double* P) {
  return guarded([&] {
    using stmg::fail;
    if (p_coarse < 1 || p_coarse > 4 || p_fine < 1 || p_fine > 4) fail(STMG_E_UNSUPPORTED, "p must be in 1..4");
    if (n_coarse < 1 || n_fine < 1 || n_fine > (1 << 20)) fail(STMG_E_ARG, "cell counts must be in 1..2^20");
    if (p_coarse > p_fine || n_fine % n_coarse != 0)
      fail(STMG_E_ARG, "the coarse space must lie in the fine one (p_coarse <= p_fine, n_coarse divides n_fine)");
    if (!rows || !cols) fail(STMG_E_ARG, "rows or cols is NULL");
    const int nf = p_fine * n_fine + 1, nc = p_coarse * n_coarse + 1;
    *rows = nf;
    *cols = nc;
    if (P) {
      if (cap < (int64_t)nf * nc) fail(STMG_E_ARG, "cap is smaller than rows * cols");
      std::fill(P, P + (size_t)nf * nc, 0.0);
      const auto L = stmg::transfer_1d_rows(p_coarse, n_coarse, p_fine, n_fine);
      for (int g = 0; g < nf; ++g)
        for (const auto& e : L[g]) P[(size_t)g * nc + e.first] = e.second;
    }
    return STMG_OK;
  });
}

stmg_status stmg_temporal_prolongation(int problem, int method, int k_fine, int c_fine, int k_coarse, int c_coarse,
                                       double slab_length, int64_t cap, int32_t* rows, int32_t* cols, double* P) {
  return guarded([&] {
    if (!(slab_length > 0.0) || !std::isfinite(slab_length)) stmg::fail(STMG_E_ARG, "slab_length must be positive");
    if (c_fine < 1 || c_coarse < 1) stmg::fail(STMG_E_ARG, "time cell counts must be >= 1");
    check_temporal(problem, method, k_fine, c_fine, slab_length / c_fine);
    check_temporal(problem, method, k_coarse, c_coarse, slab_length / c_coarse);
    if (k_coarse > k_fine || c_fine % c_coarse != 0)
      stmg::fail(STMG_E_ARG, "the coarse temporal space must lie in the fine one (k_coarse <= k_fine, c_coarse divides c_fine)");
    if (!rows || !cols) stmg::fail(STMG_E_ARG, "rows or cols is NULL");
    const stmg::hm::Temporal F = stmg::hm::temporal(problem, method, k_fine, c_fine, slab_length / c_fine);
    const stmg::hm::Temporal C = stmg::hm::temporal(problem, method, k_coarse, c_coarse, slab_length / c_coarse);
    const stmg::hm::Mat Pm = stmg::hm::temporal_prolongation(F, C);
    *rows = Pm.r;
    *cols = Pm.c;
    if (P) {
      if (cap < (int64_t)Pm.r * Pm.c) stmg::fail(STMG_E_ARG, "cap is smaller than rows * cols");
      std::copy(Pm.a.begin(), Pm.a.end(), P);
    }
    return STMG_OK;
  });
}

const char* stmg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
