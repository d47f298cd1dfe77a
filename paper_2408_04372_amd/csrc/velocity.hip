// Slab vector updates around the solve: the slab right-hand side with its coupling to the
// previous slab, and the velocity of the acoustic wave slab.
//
// Right-hand sides (Sections 2.1-2.2, eqs. heat-cg-dg-at-once, heat-cg-cg-at-once,
// wave-cg-dg-at-once, wave-cg-cg-at-once), with loads F (spatially integrated at the temporal
// DoF times), the slab vectors a = e_1 (x) alpha, b = e_1 (x) beta and g_a = A_T M_T^{-1} a,
// g_b = A_T M_T^{-1} b:
//   heat dG : (M_T (x) I) F + (a (x) M_h) u0
//   heat cGP: (M_T (x) I) F + (b (x) I) F0 - (a (x) M_h) u0 - (b (x) A_h) u0
//   wave dG : (M_T (x) I) F + (a (x) M_h) v0 + (g_a (x) M_h) u0
//   wave cGP: (M_T (x) I) F + (b (x) I) F0 - (a (x) M_h) v0 - (b (x) A_h) u0 - (g_a (x) M_h) u0
//             + (g_b (x) M_h) v0
// (the cGP coupling signs follow alpha and beta of eq. cg-time-weights), zero on Dirichlet
// nodes.  A_h u0, M_h u0 and M_h v0 come from one three-plane application of the matrix-free
// operator kernel; one node-parallel kernel combines them.
//
// Velocity of the acoustic wave slab (Sections 2.1.2 and 2.2.2, eqs. wave-cg-dg-ade and
// wave-cg-cg-ade): the first-order system's second equation gives, node by node,
//   dG(k):  V = M_T^{-1} (A_T U - a u0)
//   cGP(k): V = M_T^{-1} (A_T U + a u0 - b v0)
// with a = e_1 (x) alpha and b = e_1 (x) beta (only the first time cell couples to the
// initial data).  The n_t x n_t matrix K = M_T^{-1} A_T and the two vectors are formed on
// the host once; the kernel is one thread per lattice node (coalesced over the x-fastest
// node index in every temporal plane), HBM bound: it reads U, u0, v0 and writes V.
#include "handle.hpp"
#include "hostmath.hpp"
#include "kernels.hpp"

namespace stmg {

namespace {

constexpr int VMAX = 32;    // n_t <= 32

__global__ __launch_bounds__(256) void k_velocity(const double* __restrict__ K, const double* __restrict__ cu,
                                                  const double* __restrict__ cv, int n_t, long long nx,
                                                  const double* __restrict__ U, const double* __restrict__ u0,
                                                  const double* __restrict__ v0, double* __restrict__ V) {
  __shared__ double sK[VMAX * VMAX + 2 * VMAX];
  for (int i = threadIdx.x; i < n_t * n_t; i += blockDim.x) sK[i] = K[i];
  for (int i = threadIdx.x; i < n_t; i += blockDim.x) {
    sK[VMAX * VMAX + i] = cu[i];
    sK[VMAX * VMAX + VMAX + i] = cv[i];
  }
  __syncthreads();
  for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < nx; x += (long long)gridDim.x * blockDim.x) {
    double u[VMAX];
#pragma unroll
    for (int j = 0; j < VMAX; ++j) u[j] = j < n_t ? U[(long long)j * nx + x] : 0.0;
    const double a0 = u0 ? u0[x] : 0.0, b0 = v0 ? v0[x] : 0.0;
    for (int i = 0; i < n_t; ++i) {
      double s = sK[VMAX * VMAX + i] * a0 + sK[VMAX * VMAX + VMAX + i] * b0;
#pragma unroll
      for (int j = 0; j < VMAX; ++j)
        if (j < n_t) s += sK[i * n_t + j] * u[j];
      V[(long long)i * nx + x] = s;
    }
  }
}

// b[i][x] = sum_j MT[i][j] F[j][x] + cF0[i] F0[x] + cAu[i] Au[x] + cMu[i] Mu[x] + cMv[i] Mv[x]
__global__ __launch_bounds__(256) void k_rhs(const double* __restrict__ C, int n_t, long long nx,
                                             const unsigned char* __restrict__ mask, const double* __restrict__ F,
                                             const double* __restrict__ F0, const double* __restrict__ y3,
                                             double* __restrict__ b) {
  __shared__ double sC[VMAX * VMAX + 5 * VMAX];
  for (int i = threadIdx.x; i < n_t * n_t + 5 * n_t; i += blockDim.x) sC[i] = C[i];
  __syncthreads();
  const double* cF0 = sC + n_t * n_t;
  const double* cAu = cF0 + n_t;
  const double* cMu = cAu + n_t;
  const double* cMv = cMu + n_t;
  for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < nx; x += (long long)gridDim.x * blockDim.x) {
    if (!mask[x]) {
      for (int i = 0; i < n_t; ++i) b[(long long)i * nx + x] = 0.0;
      continue;
    }
    double f[VMAX];
#pragma unroll
    for (int j = 0; j < VMAX; ++j) f[j] = (F && j < n_t) ? F[(long long)j * nx + x] : 0.0;
    const double f0 = F0 ? F0[x] : 0.0;
    const double au = y3[x], mu = y3[nx + x], mv = y3[2 * nx + x];
    for (int i = 0; i < n_t; ++i) {
      double acc = cF0[i] * f0 + cAu[i] * au + cMu[i] * mu + cMv[i] * mv;
#pragma unroll
      for (int j = 0; j < VMAX; ++j)
        if (j < n_t) acc += sC[i * n_t + j] * f[j];
      b[(long long)i * nx + x] = acc;
    }
  }
}

}  // namespace

void slab_rhs(stmg_handle* h, const double* F, const double* F0, const double* u0, const double* v0, double* b) {
  const hm::Temporal& tm = h->tm;
  const int n = tm.n_t, nc = tm.nt_cell;
  if (n > VMAX) fail(STMG_E_UNSUPPORTED, "more than 32 temporal DoFs");
  hipStream_t s = h->stream;
  Level& L = *h->levels[0];
  const long long nx = L.g.nx;
  if (h->rhsc.bytes() == 0) {
    const bool dg = h->cfg.time_method == STMG_DG, heat = h->cfg.problem == STMG_HEAT;
    std::vector<double> a(n, 0.0), bb(n, 0.0);
    for (int i = 0; i < nc; ++i) { a[i] = tm.alpha[i]; bb[i] = tm.beta[i]; }
    hm::Mat Mi = hm::inverse(tm.M_T);
    auto gvec = [&](const std::vector<double>& v) {   // A_T M_T^{-1} v
      std::vector<double> w(n, 0.0), g(n, 0.0);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) w[i] += Mi(i, j) * v[j];
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) g[i] += tm.A_T(i, j) * w[j];
      return g;
    };
    std::vector<double> ga = gvec(a), gb = gvec(bb);
    std::vector<double> C((size_t)n * n + 5 * n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) C[(size_t)i * n + j] = tm.M_T(i, j);
    double* cF0 = C.data() + (size_t)n * n;
    double *cAu = cF0 + n, *cMu = cAu + n, *cMv = cMu + n;
    for (int i = 0; i < n; ++i) {
      if (heat && dg) cMu[i] = a[i];
      else if (heat) { cF0[i] = bb[i]; cMu[i] = -a[i]; cAu[i] = -bb[i]; }
      else if (dg) { cMv[i] = a[i]; cMu[i] = ga[i]; }
      else { cF0[i] = bb[i]; cMv[i] = -a[i] + gb[i]; cAu[i] = -bb[i]; cMu[i] = -ga[i]; }
    }
    h->rhsc = upload(C, s);
    // three planes: (A u0, M u0, M v0) from one operator application
    hm::Mat Mp(3, 3), Np(3, 3);
    Mp(0, 0) = 1.0;
    Np(1, 1) = 1.0;
    Np(2, 2) = 1.0;
    h->rhs_mnnz = upload_csr<double>(Mp, h->rhs_mp, h->rhs_mc, h->rhs_mv, s);
    h->rhs_nnnz = upload_csr<double>(Np, h->rhs_np, h->rhs_nc, h->rhs_nv, s);
    h->rhs3x.alloc(sizeof(double) * 3 * nx);
    h->rhs3y.alloc(sizeof(double) * 3 * nx);
  }
  TemporalDev<double> tp3;
  tp3.n_t = 3;
  tp3.mnnz = h->rhs_mnnz;
  tp3.nnnz = h->rhs_nnnz;
  tp3.mptr = h->rhs_mp.as<int>(); tp3.mcol = h->rhs_mc.as<int>(); tp3.mval = h->rhs_mv.as<double>();
  tp3.nptr = h->rhs_np.as<int>(); tp3.ncol = h->rhs_nc.as<int>(); tp3.nval = h->rhs_nv.as<double>();
  double* x3 = h->rhs3x.as<double>();
  double* y3 = h->rhs3y.as<double>();
  if (u0) { copy<double>(u0, x3, nx, s); copy<double>(u0, x3 + nx, nx, s); }
  else fill<double>(x3, 0.0, 2 * nx, s);
  if (v0) copy<double>(v0, x3 + 2 * nx, nx, s);
  else fill<double>(x3 + 2 * nx, 0.0, nx, s);
  fill<double>(y3, 0.0, 3 * nx, s);
  st_apply<double>(L.g, L.lt, tp3, x3, y3, 1.0, s);
  long long blocks = (nx + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_rhs, dim3((unsigned)blocks), dim3(256), 0, s, h->rhsc.as<double>(), n, nx,
                     L.mask.as<unsigned char>(), F, F0, y3, b);
  STMG_CHECK_LAUNCH();
}

void wave_velocity(stmg_handle* h, const double* U, const double* u0, const double* v0, double* V) {
  const hm::Temporal& tm = h->tm;
  const int n = tm.n_t;
  if (n > VMAX) fail(STMG_E_UNSUPPORTED, "more than 32 temporal DoFs");
  if (h->vel.bytes() == 0) {
    hm::Mat Mi = hm::inverse(tm.M_T);
    hm::Mat K = hm::matmul(Mi, tm.A_T);
    const int nc = tm.nt_cell;
    const bool dg = h->cfg.time_method == STMG_DG;
    std::vector<double> host((size_t)n * n + 2 * n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) host[(size_t)i * n + j] = K(i, j);
    for (int i = 0; i < n; ++i) {
      double ka = 0.0, kb = 0.0;            // (M_T^{-1} a)_i, (M_T^{-1} b)_i
      for (int j = 0; j < nc; ++j) { ka += Mi(i, j) * tm.alpha[j]; kb += Mi(i, j) * tm.beta[j]; }
      host[(size_t)n * n + i] = dg ? -ka : ka;
      host[(size_t)n * n + n + i] = dg ? 0.0 : -kb;
    }
    h->vel = upload(host, h->stream);
  }
  const double* d = h->vel.as<double>();
  const long long nx = h->levels[0]->g.nx;
  long long blocks = (nx + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_velocity, dim3((unsigned)blocks), dim3(256), 0, h->stream, d, d + (size_t)n * n,
                     d + (size_t)n * n + n, n, nx, U, u0, v0, V);
  STMG_CHECK_LAUNCH();
}

}  // namespace stmg
