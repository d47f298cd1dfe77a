// Matrix-free space-time operator  y += scale * (M_T (x) A_h + N_T (x) M_h) x  on
// interior rows (Section 3.1: S = sum_c P_c^T B_c^T D_c B_c P_c with sum
// factorisation; the temporal factors are small dense matrices and A_h u^i,
// M_h u^i are formed once per temporal DoF and reused).
//
// MI355X mapping.  A workgroup covers every output temporal DoF of a few cells in
// one round.  A "team" of p+1 lanes owns one (spatial cell, output temporal DoF i)
// pair; lane t of the team holds the
// z = t plane of the cell in registers ("XY layout": x and y sweeps are lane
// local) or, after a transpose through LDS, the y = t plane ("XZ layout": x and
// z sweeps are lane local).  The temporal mixing is done at the nodes while
// gathering: a_i = sum_j (M_T)_ij x_j feeds the stiffness, b_i = sum_j (N_T)_ij x_j
// the mass, so each team runs one fused  A_K a_i + M_K b_i  evaluation:
//   values at Gauss points by S-sweeps, reference gradients by collocation
//   D-sweeps on the Gauss points, geometry factors (per quadrature point,
//   computed once per cell into LDS), and the transposed sweeps back.
// Each cell's space-time values are staged once in LDS (coalesced loads).  With a
// per-cell buffer, one launch covers every cell and each cell writes its
// contribution to its own slot, which a node gather then sums in a fixed cell
// order; without one, cells are processed in 2^d colours of cells that share no
// node and every contribution is added with a plain read-modify-write.  Neither
// path uses atomics, so results are bitwise reproducible.  In 2D a team is a
// single lane holding the whole cell.
#include "device.hpp"
#include "kernels.hpp"

namespace stmg {

namespace {

template <class T, int N>
struct OpArgs {
  Tables<T, N> tab;
  GeomDesc g;
  TemporalDev<T> tp;
  const T* x;
  T* y;
  T* cellbuf;     // non-null: write each cell's contribution to its slot of the per-cell buffer
  T scale;
  int cpw;        // cells per workgroup
  int nblocks;
};

// Geometry factor slots per quadrature point: 3D: G00 G01 G02 G11 G12 G22 dJw; 2D: G00 G01 G11 dJw.
template <int DIM> constexpr int geo_slots() { return DIM == 3 ? 7 : 4; }

// G = rho |det J| w J^{-1} J^{-T} and |det J| w at quadrature point (qx, qy, qz) of a cell.
template <int DIM, int N>
__device__ inline void geometry(const GeomDesc& g, const double (&gq)[N], const double (&gw)[N],
                                long long cell, int cx, int cy, int cz, int qx, int qy, int qz,
                                int q, double* out) {
  double rho = g.rho ? (g.rho_q ? g.rho[cell * (long long)(DIM == 3 ? N * N * N : N * N) + q]
                                : g.rho[cell])
                     : 1.0;
  double w = gw[qx] * gw[qy] * (DIM == 3 ? gw[qz] : 1.0);
  if constexpr (DIM == 3) {
    double J[3][3];
    if (!g.verts) {
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) J[i][j] = (i == j) ? g.h[i] : 0.0;
    } else {
      double xi[3] = {gq[qx], gq[qy], gq[qz]};
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) J[i][j] = 0.0;
      const long long sy = g.nc[0] + 1, sz = (long long)(g.nc[0] + 1) * (g.nc[1] + 1);
      for (int v = 0; v < 8; ++v) {
        int b0 = v & 1, b1 = (v >> 1) & 1, b2 = (v >> 2) & 1;
        const double* X = g.verts + 3 * ((cz + b2) * sz + (cy + b1) * sy + (cx + b0));
        double n0 = b0 ? xi[0] : 1.0 - xi[0], n1 = b1 ? xi[1] : 1.0 - xi[1],
               n2 = b2 ? xi[2] : 1.0 - xi[2];
        double d0 = (b0 ? 1.0 : -1.0) * n1 * n2, d1 = n0 * (b1 ? 1.0 : -1.0) * n2,
               d2 = n0 * n1 * (b2 ? 1.0 : -1.0);
        for (int i = 0; i < 3; ++i) {
          J[i][0] += X[i] * d0;
          J[i][1] += X[i] * d1;
          J[i][2] += X[i] * d2;
        }
      }
    }
    double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    double id = 1.0 / det;
    // inverse: Jinv[i][j] = cof(J)[j][i] / det
    double Ji[3][3];
    Ji[0][0] = c00 * id;
    Ji[1][0] = c01 * id;
    Ji[2][0] = c02 * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    double s = fabs(det) * w;
    double f = rho * s;
    auto K = [&](int a, int b) { return Ji[a][0] * Ji[b][0] + Ji[a][1] * Ji[b][1] + Ji[a][2] * Ji[b][2]; };
    out[0] = f * K(0, 0);
    out[1] = f * K(0, 1);
    out[2] = f * K(0, 2);
    out[3] = f * K(1, 1);
    out[4] = f * K(1, 2);
    out[5] = f * K(2, 2);
    out[6] = s;
  } else {
    double J[2][2];
    if (!g.verts) {
      J[0][0] = g.h[0]; J[0][1] = 0.0; J[1][0] = 0.0; J[1][1] = g.h[1];
    } else {
      double xi[2] = {gq[qx], gq[qy]};
      J[0][0] = J[0][1] = J[1][0] = J[1][1] = 0.0;
      const long long sy = g.nc[0] + 1;
      for (int v = 0; v < 4; ++v) {
        int b0 = v & 1, b1 = (v >> 1) & 1;
        const double* X = g.verts + 2 * ((cy + b1) * sy + (cx + b0));
        double n0 = b0 ? xi[0] : 1.0 - xi[0], n1 = b1 ? xi[1] : 1.0 - xi[1];
        double d0 = (b0 ? 1.0 : -1.0) * n1, d1 = n0 * (b1 ? 1.0 : -1.0);
        for (int i = 0; i < 2; ++i) { J[i][0] += X[i] * d0; J[i][1] += X[i] * d1; }
      }
    }
    double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    double id = 1.0 / det;
    double Ji[2][2] = {{J[1][1] * id, -J[0][1] * id}, {-J[1][0] * id, J[0][0] * id}};
    double s = fabs(det) * w;
    double f = rho * s;
    out[0] = f * (Ji[0][0] * Ji[0][0] + Ji[0][1] * Ji[0][1]);
    out[1] = f * (Ji[0][0] * Ji[1][0] + Ji[0][1] * Ji[1][1]);
    out[2] = f * (Ji[1][0] * Ji[1][0] + Ji[1][1] * Ji[1][1]);
    out[3] = s;
  }
}

// ---- register-array sweeps on an N x N plane  A[r][c] ------------------------------
// out[r][q] = sum_c M[q][c] in[r][c]      (contract the column index)
template <class T, int N>
__device__ inline void cols(const T (&M)[N][N], const T (&in)[N][N], T (&out)[N][N]) {
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q < N; ++q) {
      T s = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) s += M[q][c] * in[r][c];
      out[r][q] = s;
    }
}
// out[r][c] = sum_q M[q][c] in[r][q]      (transposed, column index)
template <class T, int N>
__device__ inline void cols_t(const T (&M)[N][N], const T (&in)[N][N], T (&out)[N][N]) {
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int c = 0; c < N; ++c) {
      T s = 0;
#pragma unroll
      for (int q = 0; q < N; ++q) s += M[q][c] * in[r][q];
      out[r][c] = s;
    }
}
// out[q][c] = sum_r M[q][r] in[r][c]      (contract the row index)
template <class T, int N>
__device__ inline void rows(const T (&M)[N][N], const T (&in)[N][N], T (&out)[N][N]) {
#pragma unroll
  for (int q = 0; q < N; ++q)
#pragma unroll
    for (int c = 0; c < N; ++c) {
      T s = 0;
#pragma unroll
      for (int r = 0; r < N; ++r) s += M[q][r] * in[r][c];
      out[q][c] = s;
    }
}
// out[r][c] = sum_q M[q][r] in[q][c]      (transposed, row index)
template <class T, int N>
__device__ inline void rows_t(const T (&M)[N][N], const T (&in)[N][N], T (&out)[N][N]) {
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int c = 0; c < N; ++c) {
      T s = 0;
#pragma unroll
      for (int q = 0; q < N; ++q) s += M[q][r] * in[q][c];
      out[r][c] = s;
    }
}

// XY (lane t = z, A[y][x]) <-> XZ (lane t = y, A[z][x]) transpose inside one team.
template <class T, int N>
__device__ inline void xy_to_xz(T* scr, int t, const T (&in)[N][N], T (&out)[N][N]) {
#pragma unroll
  for (int y = 0; y < N; ++y)
#pragma unroll
    for (int x = 0; x < N; ++x) scr[(t * N + y) * N + x] = in[y][x];
  __syncthreads();
#pragma unroll
  for (int z = 0; z < N; ++z)
#pragma unroll
    for (int x = 0; x < N; ++x) out[z][x] = scr[(z * N + t) * N + x];
  __syncthreads();
}
template <class T, int N>
__device__ inline void xz_to_xy(T* scr, int t, const T (&in)[N][N], T (&out)[N][N]) {
#pragma unroll
  for (int z = 0; z < N; ++z)
#pragma unroll
    for (int x = 0; x < N; ++x) scr[(z * N + t) * N + x] = in[z][x];
  __syncthreads();
#pragma unroll
  for (int y = 0; y < N; ++y)
#pragma unroll
    for (int x = 0; x < N; ++x) out[y][x] = scr[(t * N + y) * N + x];
  __syncthreads();
}

// CB: write each cell's contribution to the per-cell buffer instead of adding it to y (a separate
// instantiation, so the colour path carries no code of the buffer path)
template <class T, int N, bool CB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void st_apply3(OpArgs<T, N> A,
                                                                                       ColourSet cs) {
  constexpr int NQ = N * N * N;
  constexpr int GS = 7;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n_t = A.tp.n_t;
  const int cpw = A.cpw;
  T* geo = reinterpret_cast<T*>(smem_raw);                  // [cpw][NQ][GS]
  T* xs = geo + (size_t)cpw * NQ * GS;                      // [cpw][n_t][NQ] + dummy panel: input, scratch, output
  // temporal CSR of M_T and N_T, copied to LDS so the mixing loops read no global memory
  const int mnnz = A.tp.mnnz, nnnz = A.tp.nnnz;
  T* mval_s = xs + (size_t)(cpw * n_t + 1) * NQ;
  T* nval_s = mval_s + mnnz;
  int* mptr_s = reinterpret_cast<int*>(nval_s + nnnz);
  int* nptr_s = mptr_s + n_t + 1;
  int* mcol_s = nptr_s + n_t + 1;
  int* ncol_s = mcol_s + mnnz;
  const GeomDesc& g = A.g;
  const int p = N - 1;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int team = tid / N;                                  // one team per (local cell, output i)
  const int t = tid - team * N;
  const int items = cpw * n_t;
  const long long plane = g.nx;
  const long long li0 = (long long)xcd_swizzle(blockIdx.x, A.nblocks) * cpw;
  const int ncell = (int)((cs.count - li0) < cpw ? (cs.count - li0) : cpw);

  for (int e = threadIdx.x; e < mnnz; e += blockDim.x) { mval_s[e] = A.tp.mval[e]; mcol_s[e] = A.tp.mcol[e]; }
  for (int e = threadIdx.x; e < nnnz; e += blockDim.x) { nval_s[e] = A.tp.nval[e]; ncol_s[e] = A.tp.ncol[e]; }
  for (int e = threadIdx.x; e <= n_t; e += blockDim.x) { mptr_s[e] = A.tp.mptr[e]; nptr_s[e] = A.tp.nptr[e]; }
  // geometry factors of this block's cells (the cell loop is uniform, so cell indices and vertex
  // addresses stay scalar)
  for (int lc = 0; lc < ncell; ++lc) {
    int cx, cy, cz;
    const long long cell = colour_cell(cs, g, li0 + lc, cx, cy, cz);
    for (int q = tid; q < NQ; q += nthr) {
      const int qx = q % N, qy = (q / N) % N, qz = q / (N * N);
      double o[7];
      geometry<3, N>(g, A.tab.gq, A.tab.gw, cell, cx, cy, cz, qx, qy, qz, q, o);
      T* dst = geo + ((size_t)lc * NQ + q) * GS;
#pragma unroll
      for (int s2 = 0; s2 < GS; ++s2) dst[s2] = (T)o[s2];
    }
  }
  // stage every temporal plane of the cells (Dirichlet nodes read as zero), node index fastest;
  // batches of UB loads are issued before their LDS stores, so the latencies overlap.  With at
  // least NQ threads each thread keeps one local node (offset and Dirichlet flag computed once per
  // cell) and walks the planes j0, j0 + npl, ...; otherwise the (plane, node) pairs are split flat.
  constexpr int UB = 24;
  const int total = n_t * NQ;
  const int npl = nthr >= NQ ? nthr / NQ : 0;
  const int my_node = npl ? tid % NQ : 0, my_j0 = npl ? tid / NQ : 0;
  const int mlx = my_node % N, mly = (my_node / N) % N, mlz = my_node / (N * N);
  for (int lc = 0; lc < ncell; ++lc) {
    int cx, cy, cz;
    colour_cell(cs, g, li0 + lc, cx, cy, cz);
    T* dst = xs + (size_t)lc * n_t * NQ;
    if (npl) {
      if (my_j0 >= npl) continue;
      const int gx = cx * p + mlx, gy = cy * p + mly, gz = cz * p + mlz;
      const bool in = gx != 0 && gx != g.nn[0] - 1 && gy != 0 && gy != g.nn[1] - 1 && gz != 0 &&
                      gz != g.nn[2] - 1;
      const T* src = A.x + ((long long)gz * g.nn[1] + gy) * g.nn[0] + gx;
      int jb = my_j0;
      for (; jb + (UB - 1) * npl < n_t; jb += UB * npl) {    // full batches: no per-load guard
        T v[UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) v[u] = in ? src[(long long)(jb + u * npl) * plane] : (T)0;
#pragma unroll
        for (int u = 0; u < UB; ++u) dst[(jb + u * npl) * NQ + my_node] = v[u];
      }
      for (; jb < n_t; jb += npl) dst[jb * NQ + my_node] = in ? src[(long long)jb * plane] : (T)0;
      continue;
    }
    for (int base = tid; base < total; base += UB * nthr) {
      T v[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int idx = base + u * nthr;
        v[u] = 0;
        if (idx < total) {
          const int j = idx / NQ, node = idx - j * NQ;
          const int lx = node % N, ly = (node / N) % N, lz = node / (N * N);
          const int gx = cx * p + lx, gy = cy * p + ly, gz = cz * p + lz;
          const bool in = gx != 0 && gx != g.nn[0] - 1 && gy != 0 && gy != g.nn[1] - 1 && gz != 0 &&
                          gz != g.nn[2] - 1;
          if (in) v[u] = A.x[(long long)j * plane + ((long long)gz * g.nn[1] + gy) * g.nn[0] + gx];
        }
      }
#pragma unroll
      for (int u = 0; u < UB; ++u)
        if (base + u * nthr < total) dst[base + u * nthr] = v[u];
    }
  }
  __syncthreads();

  const int lc = team / (n_t > 0 ? n_t : 1);
  const int i = team - lc * n_t;
  const bool act = team < items && lc < ncell;
  // temporal mixing from LDS: a = (M_T x)_i (stiffness input), b = (N_T x)_i (mass input); lane t = z plane
  T a[N][N], b[N][N];
#pragma unroll
  for (int y = 0; y < N; ++y)
#pragma unroll
    for (int x = 0; x < N; ++x) { a[y][x] = 0; b[y][x] = 0; }
  if (act) {
    const T* xc = xs + (size_t)lc * n_t * NQ + t * N * N;
    for (int k = mptr_s[i]; k < mptr_s[i + 1]; ++k) {
      const T c = mval_s[k];
      const T* xj = xc + (size_t)mcol_s[k] * NQ;
#pragma unroll
      for (int y = 0; y < N; ++y)
#pragma unroll
        for (int x = 0; x < N; ++x) a[y][x] += c * xj[y * N + x];
    }
    for (int k = nptr_s[i]; k < nptr_s[i + 1]; ++k) {
      const T c = nval_s[k];
      const T* xj = xc + (size_t)ncol_s[k] * NQ;
#pragma unroll
      for (int y = 0; y < N; ++y)
#pragma unroll
        for (int x = 0; x < N; ++x) b[y][x] += c * xj[y * N + x];
    }
  }
  __syncthreads();                                           // staged input no longer needed
  // the input panel of (lc, i) becomes this team's transpose scratch and finally its output;
  // lanes without an item (partial last block, lanes past the last team) use a dummy panel
  T* scr = xs + (size_t)(act ? team : items) * NQ;
  const int ts = t;

  const auto& S = A.tab.S;
  const auto& D = A.tab.D;
  T t0[N][N], t1[N][N], t2[N][N];

  // mass path: b -> values at Gauss points (x, y in XY layout, z after transpose)
  cols<T, N>(S, b, t0);                 // [y][qx]
  rows<T, N>(S, t0, b);                 // [qy][qx]
  xy_to_xz<T, N>(scr, ts, b, t0);       // lane = qy : [z][qx]
  T u[N][N];
  rows<T, N>(S, t0, u);                 // [qz][qx] values of b
  const T* gcell = geo + (size_t)(act ? lc : 0) * NQ * GS;
#pragma unroll
  for (int qz = 0; qz < N; ++qz)
#pragma unroll
    for (int qx = 0; qx < N; ++qx) u[qz][qx] *= gcell[((qz * N + ts) * N + qx) * GS + 6];

  // stiffness path: a -> values and y-derivative at Gauss points (XY), then XZ
  cols<T, N>(S, a, t0);                 // [y][qx]
  rows<T, N>(S, t0, t1);                // [qy][qx] values
  rows<T, N>(D, t1, t2);                // [qy][qx] d/dy
  xy_to_xz<T, N>(scr, ts, t1, t0);      // values  [z][qx]
  xy_to_xz<T, N>(scr, ts, t2, t1);      // dy      [z][qx]
  rows<T, N>(S, t0, a);                 // a  = values at (qx, qy=t, qz)
  rows<T, N>(S, t1, b);                 // b  = d/dy at Gauss points

  // quadrature-point operation; accumulate the x/z-derivative transposes into u
#pragma unroll
  for (int qz = 0; qz < N; ++qz)
#pragma unroll
    for (int qx = 0; qx < N; ++qx) {
      T dx = 0, dz = 0;
#pragma unroll
      for (int r = 0; r < N; ++r) {
        dx += D[qx][r] * a[qz][r];
        dz += D[qz][r] * a[r][qx];
      }
      const T dy = b[qz][qx];
      const T* G = gcell + ((qz * N + ts) * N + qx) * GS;
      const T gx = G[0] * dx + G[1] * dy + G[2] * dz;
      const T gy = G[1] * dx + G[3] * dy + G[4] * dz;
      const T gz = G[2] * dx + G[4] * dy + G[5] * dz;
      t2[qz][qx] = gy;
#pragma unroll
      for (int r = 0; r < N; ++r) {
        u[qz][r] += D[qx][r] * gx;
        u[r][qx] += D[qz][r] * gz;
      }
    }
  // integrate in z (XZ layout), then back to XY for y and x
  rows_t<T, N>(S, u, t0);               // [z][qx]
  rows_t<T, N>(S, t2, t1);              // gy integrated in z: [z][qx]
  xz_to_xy<T, N>(scr, ts, t0, u);       // lane = z: [qy][qx]
  xz_to_xy<T, N>(scr, ts, t1, t2);      // [qy][qx]
  rows_t<T, N>(D, t2, t0);              // d/dy transpose
#pragma unroll
  for (int qy = 0; qy < N; ++qy)
#pragma unroll
    for (int qx = 0; qx < N; ++qx) u[qy][qx] += t0[qy][qx];
  rows_t<T, N>(S, u, t1);               // [y][qx]
  cols_t<T, N>(S, t1, t2);              // [y][x]
  // cell output (node order) into the team's panel, then one coalesced pass over the block
  if (act) {
#pragma unroll
    for (int y = 0; y < N; ++y)
#pragma unroll
      for (int x = 0; x < N; ++x) scr[(t * N + y) * N + x] = t2[y][x];
  }
  __syncthreads();
  if constexpr (CB) {
    const long long es = ebuf_index(g, 1, 0, 0, 0, 0, 0, 0);     // plane stride of the buffer
    for (int lc2 = 0; lc2 < ncell; ++lc2) {
      int cx, cy, cz;
      colour_cell(cs, g, li0 + lc2, cx, cy, cz);
      const T* src = xs + (size_t)lc2 * n_t * NQ;
      if (npl) {
        if (my_j0 >= npl) continue;
        T* dst = A.cellbuf + ebuf_index(g, 0, cx, cy, cz, mlx, mly, mlz);
        for (int j = my_j0; j < n_t; j += npl) dst[j * es] = A.scale * src[j * NQ + my_node];
        continue;
      }
      for (int idx = tid; idx < n_t * NQ; idx += nthr) {
        const int j = idx / NQ, node = idx - j * NQ;
        const int lx = node % N, ly = (node / N) % N, lz = node / (N * N);
        A.cellbuf[ebuf_index(g, j, cx, cy, cz, lx, ly, lz)] = A.scale * src[idx];
      }
    }
    return;
  }
  if (npl) {
    // one local node per thread, as in the staging
    if (my_j0 >= npl) return;
    for (int lc2 = 0; lc2 < ncell; ++lc2) {
      int cx, cy, cz;
      colour_cell(cs, g, li0 + lc2, cx, cy, cz);
      const int gx = cx * p + mlx, gy = cy * p + mly, gz = cz * p + mlz;
      const bool in = gx != 0 && gx != g.nn[0] - 1 && gy != 0 && gy != g.nn[1] - 1 && gz != 0 &&
                      gz != g.nn[2] - 1;
      if (!in) continue;
      T* dst = A.y + ((long long)gz * g.nn[1] + gy) * g.nn[0] + gx;
      const T* src = xs + (size_t)lc2 * n_t * NQ + my_node;
      int jb = my_j0;
      for (; jb + (UB - 1) * npl < n_t; jb += UB * npl) {    // full batches: no per-load guard
        T v[UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) v[u] = dst[(long long)(jb + u * npl) * plane];
#pragma unroll
        for (int u = 0; u < UB; ++u) dst[(long long)(jb + u * npl) * plane] = v[u] + A.scale * src[(jb + u * npl) * NQ];
      }
      for (; jb < n_t; jb += npl) dst[(long long)jb * plane] += A.scale * src[jb * NQ];
    }
    return;
  }
  for (int lc2 = 0; lc2 < ncell; ++lc2) {
    int cx, cy, cz;
    colour_cell(cs, g, li0 + lc2, cx, cy, cz);
    const T* src = xs + (size_t)lc2 * n_t * NQ;
    for (int base = tid; base < total; base += UB * nthr) {
      long long addr[UB];
      T v[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int idx = base + u * nthr;
        addr[u] = -1;
        v[u] = 0;
        if (idx < total) {
          const int j = idx / NQ, node = idx - j * NQ;
          const int lx = node % N, ly = (node / N) % N, lz = node / (N * N);
          const int gx = cx * p + lx, gy = cy * p + ly, gz = cz * p + lz;
          const bool in = gx != 0 && gx != g.nn[0] - 1 && gy != 0 && gy != g.nn[1] - 1 && gz != 0 &&
                          gz != g.nn[2] - 1;
          if (in) {
            addr[u] = (long long)j * plane + ((long long)gz * g.nn[1] + gy) * g.nn[0] + gx;
            v[u] = A.y[addr[u]];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < UB; ++u)
        if (addr[u] >= 0) A.y[addr[u]] = v[u] + A.scale * src[base + u * nthr];
    }
  }
}

template <class T, int N>
__global__ __launch_bounds__(64) void st_apply2(OpArgs<T, N> A, ColourSet cs) {
  constexpr int NQ = N * N;
  constexpr int GS = 4;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* geo = reinterpret_cast<T*>(smem_raw);                  // [cpw][NQ][GS]
  const GeomDesc& g = A.g;
  const int p = N - 1;
  const int lane = threadIdx.x;
  const long long li0 = (long long)xcd_swizzle(blockIdx.x, A.nblocks) * A.cpw;
  for (int idx = lane; idx < A.cpw * NQ; idx += 64) {
    int lc = idx / NQ, q = idx - lc * NQ;
    if (li0 + lc >= cs.count) continue;
    int cx, cy, cz;
    long long cell = colour_cell(cs, g, li0 + lc, cx, cy, cz);
    double o[7];
    geometry<2, N>(g, A.tab.gq, A.tab.gw, cell, cx, cy, 0, q % N, q / N, 0, q, o);
    T* dst = geo + ((size_t)lc * NQ + q) * GS;
#pragma unroll
    for (int s = 0; s < GS; ++s) dst[s] = (T)o[s];
  }
  __syncthreads();
  const int n_t = A.tp.n_t;
  const int items = A.cpw * n_t;
  const long long plane = g.nx;
  for (int it0 = 0; it0 < items; it0 += 64) {
    const int item = it0 + lane;
    const int lc = item / n_t;
    const int i = item - lc * n_t;
    if (item >= items || li0 + lc >= cs.count) continue;
    int cx, cy, cz;
    colour_cell(cs, g, li0 + lc, cx, cy, cz);
    long long base = (long long)cy * p * g.nn[0] + (long long)cx * p;
    bool inner[N][N];
#pragma unroll
    for (int y = 0; y < N; ++y)
#pragma unroll
      for (int x = 0; x < N; ++x) {
        int gy = cy * p + y, gx = cx * p + x;
        inner[y][x] = gy != 0 && gy != g.nn[1] - 1 && gx != 0 && gx != g.nn[0] - 1;
      }
    T a[N][N], b[N][N];
#pragma unroll
    for (int y = 0; y < N; ++y)
#pragma unroll
      for (int x = 0; x < N; ++x) { a[y][x] = 0; b[y][x] = 0; }
    for (int k = A.tp.mptr[i]; k < A.tp.mptr[i + 1]; ++k) {
      const T c = A.tp.mval[k];
      const T* xj = A.x + (long long)A.tp.mcol[k] * plane + base;
#pragma unroll
      for (int y = 0; y < N; ++y)
#pragma unroll
        for (int x = 0; x < N; ++x)
          if (inner[y][x]) a[y][x] += c * xj[(long long)y * g.nn[0] + x];
    }
    for (int k = A.tp.nptr[i]; k < A.tp.nptr[i + 1]; ++k) {
      const T c = A.tp.nval[k];
      const T* xj = A.x + (long long)A.tp.ncol[k] * plane + base;
#pragma unroll
      for (int y = 0; y < N; ++y)
#pragma unroll
        for (int x = 0; x < N; ++x)
          if (inner[y][x]) b[y][x] += c * xj[(long long)y * g.nn[0] + x];
    }
    const auto& S = A.tab.S;
    const auto& D = A.tab.D;
    T t0[N][N], ah[N][N], bh[N][N], gx[N][N], gy[N][N];
    cols<T, N>(S, a, t0);
    rows<T, N>(S, t0, ah);      // [qy][qx]
    cols<T, N>(S, b, t0);
    rows<T, N>(S, t0, bh);
    const T* gcell = geo + (size_t)lc * NQ * GS;
#pragma unroll
    for (int qy = 0; qy < N; ++qy)
#pragma unroll
      for (int qx = 0; qx < N; ++qx) {
        T dx = 0, dy = 0;
#pragma unroll
        for (int r = 0; r < N; ++r) {
          dx += D[qx][r] * ah[qy][r];
          dy += D[qy][r] * ah[r][qx];
        }
        const T* G = gcell + (qy * N + qx) * GS;
        gx[qy][qx] = G[0] * dx + G[1] * dy;
        gy[qy][qx] = G[1] * dx + G[2] * dy;
        bh[qy][qx] *= G[3];
      }
    cols_t<T, N>(D, gx, t0);
    rows_t<T, N>(D, gy, ah);
#pragma unroll
    for (int qy = 0; qy < N; ++qy)
#pragma unroll
      for (int qx = 0; qx < N; ++qx) bh[qy][qx] += t0[qy][qx] + ah[qy][qx];
    rows_t<T, N>(S, bh, t0);    // [y][qx]
    cols_t<T, N>(S, t0, ah);    // [y][x]
    if (A.cellbuf) {
#pragma unroll
      for (int y = 0; y < N; ++y)
#pragma unroll
        for (int x = 0; x < N; ++x) A.cellbuf[ebuf_index(g, i, cx, cy, 0, x, y, 0)] = A.scale * ah[y][x];
      continue;
    }
    T* yi = A.y + (long long)i * plane + base;
#pragma unroll
    for (int y = 0; y < N; ++y)
#pragma unroll
      for (int x = 0; x < N; ++x)
        if (inner[y][x]) yi[(long long)y * g.nn[0] + x] += A.scale * ah[y][x];
  }
}

template <class T, int N>
Tables<T, N> make_tables(const LevelTables& lt) {
  Tables<T, N> tb;
  for (int q = 0; q < N; ++q) {
    tb.gq[q] = lt.gq[q];
    tb.gw[q] = lt.gw[q];
    for (int i = 0; i < N; ++i) {
      tb.S[q][i] = (T)lt.S[q * N + i];
      tb.D[q][i] = (T)lt.D[q * N + i];
    }
  }
  return tb;
}

// cells per workgroup: fill the teams of one wave as evenly as possible
int pick_cpw(int teams, int n_t) {
  int best = 1;
  double be = -1.0;
  for (int c = 1; c <= 16; ++c) {
    int items = c * n_t;
    int rounds = (items + teams - 1) / teams;
    double eff = (double)items / (rounds * teams);
    if (eff > be + 1e-9) { be = eff; best = c; }
    if (items >= 4 * teams) break;
  }
  return best;
}

template <class T, int N>
void launch_apply(const GeomDesc& g, const LevelTables& lt, const TemporalDev<T>& tp,
                  const T* x, T* y, T scale, hipStream_t s, T* cellbuf, const T* base, bool overwrite) {
  OpArgs<T, N> A;
  A.tab = make_tables<T, N>(lt);
  A.g = g;
  A.tp = tp;
  A.x = x;
  A.y = y;
  A.cellbuf = cellbuf;
  A.scale = scale;
  size_t lds;
  int threads = 64;
  if (g.dim == 3) {
    constexpr int NQ = N * N * N;
    // all n_t outputs of cpw cells in one round: cpw * n_t teams of N lanes, at most 256 lanes
    int per_cell = N * tp.n_t;
    if (per_cell > 256) fail(STMG_E_UNSUPPORTED, "too many temporal DoFs for the operator kernel");
    const size_t csr = sizeof(T) * (size_t)(tp.mnnz + tp.nnnz) + sizeof(int) * (size_t)(2 * (tp.n_t + 1) + tp.mnnz + tp.nnnz);
    int best = 1;
    double be = -1.0;
    for (int c = 1; c * per_cell <= 256; ++c) {
      int lanes = c * per_cell;
      int th = (lanes + 63) / 64 * 64;
      double eff = (double)lanes / th;
      size_t l = sizeof(T) * ((size_t)c * NQ * (7 + tp.n_t) + NQ) + csr;
      if (l > 64 * 1024) break;
      if (eff > be + 1e-9) { be = eff; best = c; }
    }
    A.cpw = best;
    threads = (A.cpw * per_cell + 63) / 64 * 64;
    lds = sizeof(T) * ((size_t)A.cpw * NQ * (7 + tp.n_t) + NQ) + csr;
  } else {
    constexpr int NQ = N * N;
    A.cpw = pick_cpw(64, tp.n_t);
    lds = sizeof(T) * ((size_t)A.cpw * NQ * 4);
  }
  const int nsets = cellbuf ? 1 : n_colours(g.dim);
  for (int colour = 0; colour < nsets; ++colour) {
    ColourSet cs = cellbuf ? all_cells(g) : colour_set(g, colour);
    if (cs.count == 0) continue;
    A.nblocks = ceil_div(cs.count, A.cpw);
    if (g.dim == 3) {
      if (cellbuf) hipLaunchKernelGGL((st_apply3<T, N, true>), dim3(A.nblocks), dim3(threads), lds, s, A, cs);
      else hipLaunchKernelGGL((st_apply3<T, N, false>), dim3(A.nblocks), dim3(threads), lds, s, A, cs);
    }
    else hipLaunchKernelGGL((st_apply2<T, N>), dim3(A.nblocks), dim3(64), lds, s, A, cs);
    STMG_CHECK_LAUNCH();
  }
  if (cellbuf) cell_gather<T>(g, tp.n_t, cellbuf, y, s, base, overwrite);
}

}  // namespace

template <class T>
void st_apply(const GeomDesc& g, const LevelTables& lt, const TemporalDev<T>& tp, const T* x, T* y,
              T scale, hipStream_t s, T* cellbuf, const T* base, bool overwrite) {
  if (overwrite && !cellbuf) fail(STMG_E_UNSUPPORTED, "overwrite needs the per-cell buffer");
  if (g.ncells == 0 || tp.n_t == 0) return;
  switch (g.n) {
    case 2: launch_apply<T, 2>(g, lt, tp, x, y, scale, s, cellbuf, base, overwrite); break;
    case 3: launch_apply<T, 3>(g, lt, tp, x, y, scale, s, cellbuf, base, overwrite); break;
    case 4: launch_apply<T, 4>(g, lt, tp, x, y, scale, s, cellbuf, base, overwrite); break;
    case 5: launch_apply<T, 5>(g, lt, tp, x, y, scale, s, cellbuf, base, overwrite); break;
    default: fail(STMG_E_UNSUPPORTED, "p must be 1..4");
  }
}

template void st_apply<double>(const GeomDesc&, const LevelTables&, const TemporalDev<double>&,
                               const double*, double*, double, hipStream_t, double*, const double*, bool);
template void st_apply<float>(const GeomDesc&, const LevelTables&, const TemporalDev<float>&,
                              const float*, float*, float, hipStream_t, float*, const float*, bool);

}  // namespace stmg
