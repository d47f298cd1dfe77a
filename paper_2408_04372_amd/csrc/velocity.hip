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

}  // namespace

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
