// Device-side descriptors shared by the kernels: one level's spatial
// discretisation and the slab's temporal factors.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace stmg {

constexpr int MAXN = 5;   // p + 1 <= 5

// Spatial discretisation of one level (lattice of Q_p cells).
struct GeomDesc {
  int dim = 3, p = 1, n = 2;
  int nc[3] = {1, 1, 1};   // cells per direction
  int nn[3] = {1, 1, 1};   // nodes per direction
  long long nx = 1;        // nodes per temporal plane
  long long ncells = 1;
  const double* verts = nullptr;   // vertex lattice (nc+1)^dim x dim, or null (Cartesian)
  double lo[3] = {0, 0, 0}, h[3] = {1, 1, 1};
  const double* rho = nullptr;     // per cell, or per (cell, quadrature point) if rho_q
  int rho_q = 0;
};

// Slab temporal factors in CSR form (rows i, columns j), device pointers.
template <class T>
struct TemporalDev {
  int n_t = 0;
  int mnnz = 0, nnnz = 0;   // stored entries of M_T and N_T
  const int* mptr = nullptr; const int* mcol = nullptr; const T* mval = nullptr;
  const int* nptr = nullptr; const int* ncol = nullptr; const T* nval = nullptr;
  // union pattern of M_T and N_T with both values per entry (zero where one of them has none)
  int unnz = 0;
  const int* uptr = nullptr; const int* ucol = nullptr; const T* umval = nullptr; const T* unval = nullptr;
};

// 1D tables of Q_p with GLL nodes at the (p+1)-point Gauss rule:
// S[q][i] = l_i(xi_q), D[q][r] = l^G_r'(xi_q) (collocation derivative on the Gauss points).
template <class T, int N>
struct Tables {
  T S[N][N];
  T D[N][N];
  double gq[N];   // Gauss points on [0, 1]
  double gw[N];   // Gauss weights
};

// XCD-aware block order: consecutive logical blocks land on the same XCD
// (hardware dispatches workgroups round-robin over the 8 XCDs).
__device__ inline int xcd_swizzle(int b, int nb) {
  int per = nb >> 3, rem = nb & 7, xcd = b & 7, idx = b >> 3;
  return (xcd < rem) ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

template <class T> __device__ inline void atomic_add(T* p, T v) { unsafeAtomicAdd(p, v); }

// Cells of one colour (cx % 2, cy % 2, cz % 2) = (colour & 1, colour >> 1 & 1, colour >> 2 & 1)
// share no lattice node, so a launch over one colour may update its nodes without atomics.
struct ColourSet {
  int colour = 0;
  int step = 2;           // 2: one colour (every other cell per direction); 1: every cell
  int m[3] = {1, 1, 1};   // cells of this parity per direction
  long long count = 0;
};
inline ColourSet colour_set(const GeomDesc& g, int colour) {
  ColourSet c;
  c.colour = colour;
  c.count = 1;
  for (int d = 0; d < 3; ++d) {
    int o = (colour >> d) & 1;
    c.m[d] = (d < g.dim) ? (g.nc[d] - o + 1) / 2 : (o ? 0 : 1);
    c.count *= c.m[d];
  }
  return c;
}
// every cell in one set (used with per-cell output buffers, where no two cells write one node)
inline ColourSet all_cells(const GeomDesc& g) {
  ColourSet c;
  c.step = 1;
  c.count = 1;
  for (int d = 0; d < 3; ++d) {
    c.m[d] = (d < g.dim) ? g.nc[d] : 1;
    c.count *= c.m[d];
  }
  return c;
}
__device__ inline long long colour_cell(const ColourSet& cs, const GeomDesc& g, long long li, int& cx,
                                        int& cy, int& cz) {
  int ix = (int)(li % cs.m[0]);
  long long r = li / cs.m[0];
  int iy = (int)(r % cs.m[1]);
  int iz = (int)(r / cs.m[1]);
  const int c = cs.step == 2 ? cs.colour : 0;
  cx = cs.step * ix + (c & 1);
  cy = cs.step * iy + ((c >> 1) & 1);
  cz = cs.step * iz + ((c >> 2) & 1);
  return ((long long)cz * g.nc[1] + cy) * g.nc[0] + cx;
}
inline int n_colours(int dim) { return dim == 3 ? 8 : 4; }

// Per-cell buffer: every cell keeps its own copy of its n^d local nodes, temporal plane slowest.
// For n >= 4 each cell's n^d values of a plane are contiguous ([plane][cell][local node]), so a
// cell writes whole cache lines; for smaller cells the copies form a "broken lattice" of nc * n
// points per direction (cell c, local node l at c * n + l), where neighbouring cells write
// neighbouring runs and the gather reads consecutive positions for consecutive nodes.
constexpr int EBUF_CELL_MAJOR_N = 4;
__device__ inline long long ebuf_index(const GeomDesc& g, int j, int cx, int cy, int cz, int lx, int ly, int lz) {
  const int n = g.n;
  if (n >= EBUF_CELL_MAJOR_N) {
    const long long nq = g.dim == 3 ? (long long)n * n * n : (long long)n * n;
    const long long cell = ((long long)cz * g.nc[1] + cy) * g.nc[0] + cx;
    return ((long long)j * g.ncells + cell) * nq + ((long long)lz * n + ly) * n + lx;
  }
  const long long ex = (long long)g.nc[0] * n, ey = (long long)g.nc[1] * n;
  const long long ez = g.dim == 3 ? (long long)g.nc[2] * n : 1;
  const long long zz = g.dim == 3 ? (long long)cz * n + lz : 0;
  return (((long long)j * ez + zz) * ey + (long long)cy * n + ly) * ex + (long long)cx * n + lx;
}

}  // namespace stmg
