// Separable vertex-patch variant of the space-time additive Schwarz smoother: the extension of
// the cell-wise smoother that Section 5 names for robustness in the polynomial degree, built on
// the cheaper (fast diagonalisation) inner solver.  One block per interior vertex v of the cell
// lattice: the lattice nodes strictly inside the 2^d cells around v (2p - 1 per axis) times the
// temporal DoFs of one time cell.  On a Cartesian level the patch operator with the mean
// coefficient rho_v of its cells is a Kronecker product of the assembled 1D two-cell matrices
// restricted to the 2p - 1 inner nodes, the same for every patch of the level:
//   M~ = M_z (x) M_y (x) M_x,  A~ = rho_v (A_z (x) M_y (x) M_x + M_z (x) A_y (x) M_x + M_z (x) M_y (x) A_x).
// With A_a Q_a = M_a Q_a diag(lambda_a), Q_a^T M_a Q_a = I, the block inverse is
//   (I (x) Q) blockdiag_s (rho_v (lambda_x + lambda_y + lambda_z)_s M_tau + N~)^{-1} (I (x) Q^T).
// Every patch node is an interior node of the domain, so no boundary cases arise.  Patches around
// vertices of one parity class (v mod 2 per axis) share no node: 2^d colour launches add
// omega * (block solve) into u without atomics, in a fixed order.
#include "kernels.hpp"

namespace stmg {

namespace {

constexpr int PATCH_MAXTC = 6;   // temporal DoFs per time cell

struct PatchSet {
  int o[3] = {1, 1, 1};          // first vertex of this parity per axis (1 or 2)
  int m[3] = {1, 1, 1};          // vertices of this parity per axis
  long long count = 0;
};

inline PatchSet patch_set(const GeomDesc& g, int colour) {
  PatchSet ps;
  ps.count = 1;
  for (int d = 0; d < 3; ++d) {
    if (d >= g.dim) {
      ps.o[d] = 0;
      ps.m[d] = (colour >> d) & 1 ? 0 : 1;
    } else {
      // interior vertices 1 .. nc - 1 with v % 2 == parity
      ps.o[d] = (colour >> d) & 1 ? 1 : 2;
      ps.m[d] = ps.o[d] <= g.nc[d] - 1 ? (g.nc[d] - 1 - ps.o[d]) / 2 + 1 : 0;
    }
    ps.count *= ps.m[d];
  }
  return ps;
}

template <class T, int DIM, int P>
__global__ __launch_bounds__(256) void k_asm_patch(GeomDesc g, PatchSet ps, int n_t, int ntc,
                                                   const T* __restrict__ pq, const T* __restrict__ pl,
                                                   const T* __restrict__ prho, const T* __restrict__ ptm,
                                                   const T* __restrict__ r, T* __restrict__ u, T omega,
                                                   int nblocks) {
  constexpr int NS = DIM == 3 ? P * P * P : P * P;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* X = reinterpret_cast<T*>(smem_raw);                 // [n_t][NS]
  __shared__ T sQ[3][P][P], sL[3][P], sTM[2][PATCH_MAXTC * PATCH_MAXTC];
  const long long li = xcd_swizzle(blockIdx.x, nblocks);
  if (li >= ps.count) return;
  const int ix = (int)(li % ps.m[0]), iy = (int)((li / ps.m[0]) % ps.m[1]),
            iz = DIM == 3 ? (int)(li / ((long long)ps.m[0] * ps.m[1])) : 0;
  const int v[3] = {ps.o[0] + 2 * ix, ps.o[1] + 2 * iy, DIM == 3 ? ps.o[2] + 2 * iz : 0};
  const int p = g.p;
  const int g0[3] = {p * (v[0] - 1) + 1, p * (v[1] - 1) + 1, DIM == 3 ? p * (v[2] - 1) + 1 : 0};
  const int tid = threadIdx.x;
  for (int idx = tid; idx < DIM * P * P; idx += blockDim.x) {
    const int a = idx / (P * P), e = idx % (P * P);
    sQ[a][e / P][e % P] = pq[a * P * P + e];
    if (e < P) sL[a][e] = pl[a * P + e];
  }
  for (int idx = tid; idx < 2 * ntc * ntc; idx += blockDim.x) sTM[idx / (ntc * ntc)][idx % (ntc * ntc)] = ptm[idx];
  const long long vi = DIM == 3 ? ((long long)(v[2] - 1) * (g.nc[1] - 1) + (v[1] - 1)) * (g.nc[0] - 1) + (v[0] - 1)
                                : (long long)(v[1] - 1) * (g.nc[0] - 1) + (v[0] - 1);
  const T rho = prho[vi];
  // stage r on the patch's nodes (all interior nodes of the domain)
  for (int idx = tid; idx < n_t * NS; idx += blockDim.x) {
    const int j = idx / NS, a = idx % NS;
    const int lx = a % P, ly = (a / P) % P, lz = DIM == 3 ? a / (P * P) : 0;
    const int gx = g0[0] + lx, gy = g0[1] + ly, gz = g0[2] + lz;
    X[idx] = r[(long long)j * g.nx + ((long long)gz * g.nn[1] + gy) * g.nn[0] + gx];
  }
  __syncthreads();
  // one 1D transform along axis `ax` of every line: forward (Q^T) or backward (Q)
  auto sweep = [&](int ax, bool forward) {
    constexpr int LINES = NS / P;
    const int stride = ax == 0 ? 1 : (ax == 1 ? P : P * P);
    for (int line = tid; line < n_t * LINES; line += blockDim.x) {
      const int j = line / LINES, l = line % LINES;
      int base;
      if (ax == 0) base = l * P;
      else if (ax == 1) base = (l % P) + (l / P) * P * P;
      else base = l;
      T* w = X + j * NS + base;
      T in[P], out[P];
#pragma unroll
      for (int k = 0; k < P; ++k) in[k] = w[k * stride];
#pragma unroll
      for (int i = 0; i < P; ++i) {
        T acc = 0;
#pragma unroll
        for (int k = 0; k < P; ++k) acc += (forward ? sQ[ax][k][i] : sQ[ax][i][k]) * in[k];
        out[i] = acc;
      }
#pragma unroll
      for (int i = 0; i < P; ++i) w[i * stride] = out[i];
    }
    __syncthreads();
  };
  for (int ax = 0; ax < DIM; ++ax) sweep(ax, true);
  // per mode s and time cell m: (rho lambda_s M_tau + N~) w = W[m, :, s], partial pivoting
  const int c = n_t / ntc;
  for (int pair = tid; pair < c * NS; pair += blockDim.x) {
    const int m = pair / NS, s = pair % NS;
    const int kx = s % P, ky = (s / P) % P, kz = DIM == 3 ? s / (P * P) : 0;
    const T lam = rho * (sL[0][kx] + sL[1][ky] + (DIM == 3 ? sL[2][kz] : (T)0));
    T A[PATCH_MAXTC][PATCH_MAXTC], b[PATCH_MAXTC];
    for (int i = 0; i < ntc; ++i) {
      b[i] = X[(m * ntc + i) * NS + s];
      for (int k = 0; k < ntc; ++k) A[i][k] = lam * sTM[0][i * ntc + k] + sTM[1][i * ntc + k];
    }
    for (int k = 0; k < ntc; ++k) {
      int piv = k;
      for (int i = k + 1; i < ntc; ++i)
        if (fabs((double)A[i][k]) > fabs((double)A[piv][k])) piv = i;
      if (piv != k) {
        for (int e = 0; e < ntc; ++e) { T t = A[k][e]; A[k][e] = A[piv][e]; A[piv][e] = t; }
        T t = b[k]; b[k] = b[piv]; b[piv] = t;
      }
      const T inv = (T)1 / A[k][k];
      for (int i = k + 1; i < ntc; ++i) {
        const T f = A[i][k] * inv;
        for (int e = k; e < ntc; ++e) A[i][e] -= f * A[k][e];
        b[i] -= f * b[k];
      }
    }
    for (int i = ntc - 1; i >= 0; --i) {
      T acc = b[i];
      for (int e = i + 1; e < ntc; ++e) acc -= A[i][e] * b[e];
      b[i] = acc / A[i][i];
    }
    for (int i = 0; i < ntc; ++i) X[(m * ntc + i) * NS + s] = b[i];
  }
  __syncthreads();
  for (int ax = DIM - 1; ax >= 0; --ax) sweep(ax, false);
  // add omega Z to the patch's nodes (patches of one colour share no node)
  for (int idx = tid; idx < n_t * NS; idx += blockDim.x) {
    const int j = idx / NS, a = idx % NS;
    const int lx = a % P, ly = (a / P) % P, lz = DIM == 3 ? a / (P * P) : 0;
    const int gx = g0[0] + lx, gy = g0[1] + ly, gz = g0[2] + lz;
    u[(long long)j * g.nx + ((long long)gz * g.nn[1] + gy) * g.nn[0] + gx] += omega * X[idx];
  }
}

template <class T, int DIM, int P>
void launch_patch(const GeomDesc& g, const PatchSet& ps, int n_t, int ntc, const T* pq, const T* pl, const T* prho,
                  const T* ptm, const T* r, T* u, T omega, hipStream_t s) {
  constexpr int NS = DIM == 3 ? P * P * P : P * P;
  const int nb = (int)ps.count;
  hipLaunchKernelGGL((k_asm_patch<T, DIM, P>), dim3(nb), dim3(256), sizeof(T) * (size_t)n_t * NS, s, g, ps, n_t,
                     ntc, pq, pl, prho, ptm, r, u, omega, nb);
}

}  // namespace

bool patch_applicable(const GeomDesc& g, int nt_cell) {
  if (g.verts || nt_cell < 1 || nt_cell > PATCH_MAXTC || g.p < 1 || g.p > 4) return false;
  for (int d = 0; d < g.dim; ++d)
    if (g.nc[d] < 2) return false;
  return true;
}

template <class T>
void asm_apply_patch(const GeomDesc& g, int n_t, int nt_cell, const T* pq, const T* pl, const T* prho, const T* ptm,
                     const T* r, T* u, T omega, hipStream_t s) {
  if (!patch_applicable(g, nt_cell)) fail(STMG_E_UNSUPPORTED, "the vertex-patch smoother needs a Cartesian level with at least two cells per direction and at most 6 temporal DoFs per time cell");
  const int P = 2 * g.p - 1;
  const long long ns = g.dim == 3 ? (long long)P * P * P : (long long)P * P;
  if ((size_t)n_t * ns * sizeof(T) > 64 * 1024) fail(STMG_E_UNSUPPORTED, "patch too large for the vertex-patch smoother");
  for (int colour = 0; colour < n_colours(g.dim); ++colour) {
    const PatchSet ps = patch_set(g, colour);
    if (ps.count == 0) continue;
    if (ps.count > (1LL << 31) - 1) fail(STMG_E_UNSUPPORTED, "too many vertex patches");
    if (g.dim == 3) {
      switch (P) {
        case 1: launch_patch<T, 3, 1>(g, ps, n_t, nt_cell, pq, pl, prho, ptm, r, u, omega, s); break;
        case 3: launch_patch<T, 3, 3>(g, ps, n_t, nt_cell, pq, pl, prho, ptm, r, u, omega, s); break;
        case 5: launch_patch<T, 3, 5>(g, ps, n_t, nt_cell, pq, pl, prho, ptm, r, u, omega, s); break;
        default: launch_patch<T, 3, 7>(g, ps, n_t, nt_cell, pq, pl, prho, ptm, r, u, omega, s); break;
      }
    } else {
      switch (P) {
        case 1: launch_patch<T, 2, 1>(g, ps, n_t, nt_cell, pq, pl, prho, ptm, r, u, omega, s); break;
        case 3: launch_patch<T, 2, 3>(g, ps, n_t, nt_cell, pq, pl, prho, ptm, r, u, omega, s); break;
        case 5: launch_patch<T, 2, 5>(g, ps, n_t, nt_cell, pq, pl, prho, ptm, r, u, omega, s); break;
        default: launch_patch<T, 2, 7>(g, ps, n_t, nt_cell, pq, pl, prho, ptm, r, u, omega, s); break;
      }
    }
    STMG_CHECK_LAUNCH();
  }
}

template void asm_apply_patch<double>(const GeomDesc&, int, int, const double*, const double*, const double*,
                                      const double*, const double*, double*, double, hipStream_t);
template void asm_apply_patch<float>(const GeomDesc&, int, int, const float*, const float*, const float*,
                                     const float*, const float*, float*, float, hipStream_t);

}  // namespace stmg
