// Node coordinates and point values of the finest-level Q_p field (Cartesian meshes), used
// to set initial data and to evaluate point goal quantities such as the displacement at
// fixed locations of the structural-health-monitoring example (Section 4.2).
//
// A point x lies in cell c = floor((x - lo) / h) (clamped to the mesh) at reference
// coordinate xi = (x - lo) / h - c; its value is sum_b u_b prod_d l_{b_d}(xi_d) with the 1D
// Lagrange basis on the Gauss-Lobatto nodes.  The host forms the node offsets and weights
// of every point; one kernel sums them for every requested temporal plane.
#include "handle.hpp"
#include "hostmath.hpp"
#include "kernels.hpp"

namespace stmg {

namespace {

// out[t][q] = sum_b w[q][b] U[t][off[q][b]]   (nb = (p+1)^d weights per point)
__global__ void k_points(const double* __restrict__ U, long long nx, int n_planes, int npts, int nb,
                         const long long* __restrict__ off, const double* __restrict__ w,
                         double* __restrict__ out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_planes * npts) return;
  const int t = idx / npts, q = idx % npts;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += w[(size_t)q * nb + b] * U[(long long)t * nx + off[(size_t)q * nb + b]];
  out[idx] = s;
}

void require_cartesian(const stmg_handle* h) {
  if (h->levels[0]->g.verts) fail(STMG_E_UNSUPPORTED, "node coordinates and point values need a Cartesian mesh");
}

}  // namespace

void node_coordinates(stmg_handle* h, double* xyz) {
  require_cartesian(h);
  const GeomDesc& g = h->levels[0]->g;
  const int d = g.dim, p = g.p;
  hm::Vec gl = hm::gauss_lobatto(p + 1);
  std::vector<double> c1[3];
  for (int a = 0; a < d; ++a) {
    const double hx = (h->cfg.hi[a] - h->cfg.lo[a]) / g.nc[a];
    c1[a].resize(g.nn[a]);
    for (int i = 0; i < g.nn[a]; ++i) {
      const int cell = std::min(i / p, g.nc[a] - 1), l = i - cell * p;
      c1[a][i] = h->cfg.lo[a] + (cell + gl[l]) * hx;
    }
  }
  for (long long n = 0; n < g.nx; ++n) {
    long long r = n;
    for (int a = 0; a < d; ++a) {
      xyz[n * d + a] = c1[a][r % g.nn[a]];
      r /= g.nn[a];
    }
  }
}

void point_values(stmg_handle* h, const double* U, int n_planes, int npts, const double* pts, double* out) {
  require_cartesian(h);
  const GeomDesc& g = h->levels[0]->g;
  const int d = g.dim, p = g.p, n = p + 1;
  const int nb = d == 3 ? n * n * n : n * n;
  hm::Vec gl = hm::gauss_lobatto(n);
  std::vector<long long> off((size_t)npts * nb);
  std::vector<double> w((size_t)npts * nb);
  for (int q = 0; q < npts; ++q) {
    int cell[3] = {0, 0, 0};
    hm::Mat V[3];
    for (int a = 0; a < d; ++a) {
      const double lo = h->cfg.lo[a], hi = h->cfg.hi[a], x = pts[(size_t)q * d + a];
      if (!(x >= lo && x <= hi)) fail(STMG_E_ARG, "point " + std::to_string(q) + " lies outside the domain");
      const double hx = (hi - lo) / g.nc[a];
      cell[a] = std::min((int)std::floor((x - lo) / hx), g.nc[a] - 1);
      const double xi = (x - lo) / hx - cell[a];
      hm::Mat D;
      hm::lagrange(gl, hm::Vec{xi}, V[a], D);
    }
    for (int b = 0; b < nb; ++b) {
      const int lx = b % n, ly = (b / n) % n, lz = d == 3 ? b / (n * n) : 0;
      const long long gx = (long long)cell[0] * p + lx, gy = (long long)cell[1] * p + ly,
                      gz = d == 3 ? (long long)cell[2] * p + lz : 0;
      off[(size_t)q * nb + b] = (gz * g.nn[1] + gy) * g.nn[0] + gx;
      w[(size_t)q * nb + b] = V[0](0, lx) * V[1](0, ly) * (d == 3 ? V[2](0, lz) : 1.0);
    }
  }
  hipStream_t s = h->stream;
  DevBuf doff = upload(off, s), dw = upload(w, s), dout(sizeof(double) * (size_t)n_planes * npts);
  const int total = n_planes * npts;
  hipLaunchKernelGGL(k_points, dim3((total + 255) / 256), dim3(256), 0, s, U, g.nx, n_planes, npts, nb,
                     doff.as<long long>(), dw.as<double>(), dout.as<double>());
  STMG_CHECK_LAUNCH();
  std::vector<double> o = download<double>(dout.get(), (size_t)total, s);
  std::copy(o.begin(), o.end(), out);
}

}  // namespace stmg
