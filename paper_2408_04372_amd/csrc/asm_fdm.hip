// Separable (fast diagonalisation) variant of the space-time cell-wise additive Schwarz
// smoother (Section 3.3, eqs. vanka0, vanka; a cheaper local solver in the sense of the
// paper's outlook).  On a Cartesian cell the spatial blocks are replaced by Kronecker
// products of per-axis principal submatrices of the assembled 1D matrices,
//   M~ = M_z (x) M_y (x) M_x,  A~ = rho_K (A_z (x) M_y (x) M_x + M_z (x) A_y (x) M_x + M_z (x) M_y (x) A_x),
// exact when the coefficient is constant.  With the 1D generalised eigenpairs
// A_d Q_d = M_d Q_d diag(lambda_d), Q_d^T M_d Q_d = I, the block inverse is
//   (I (x) Q) blockdiag_s (rho_K (lambda_x + lambda_y + lambda_z)_s M_tau + N~)^{-1} (I (x) Q^T),
// Q = Q_z (x) Q_y (x) Q_x.  Per cell: d sum-factorisation sweeps forward, one small temporal
// solve per mode and time cell, d sweeps back.  Nothing per cell is stored except rho_K; the
// 1D tables depend only on the axis and on whether the cell touches the lower / upper
// boundary along it (Dirichlet nodes are decoupled identity rows, masked on input and output).
#include "kernels.hpp"

namespace stmg {

namespace {

constexpr int FDM_MAXTC = 6;    // temporal DoFs per time cell

template <class T, int DIM, int N>
__global__ __launch_bounds__(256) void k_asm_fdm(GeomDesc g, ColourSet cs, int n_t, int ntc, const T* __restrict__ fq,
                                                 const T* __restrict__ fl, const T* __restrict__ frho,
                                                 const T* __restrict__ ftm, const T* __restrict__ r,
                                                 T* __restrict__ u, T omega, int nblocks, T* __restrict__ cellbuf) {
  constexpr int NS = DIM == 3 ? N * N * N : N * N;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* X = reinterpret_cast<T*>(smem_raw);                 // [n_t][NS]
  __shared__ T sQ[3][N][N], sL[3][N], sTM[2][FDM_MAXTC * FDM_MAXTC];
  const long long li = xcd_swizzle(blockIdx.x, nblocks);
  if (li >= cs.count) return;
  int cc[3];
  const long long cell = colour_cell(cs, g, li, cc[0], cc[1], cc[2]);
  const int tid = threadIdx.x;
  for (int idx = tid; idx < DIM * N * N; idx += blockDim.x) {
    const int a = idx / (N * N), e = idx % (N * N);
    const int bc = (cc[a] == 0 ? 1 : 0) + (cc[a] == g.nc[a] - 1 ? 2 : 0);
    sQ[a][e / N][e % N] = fq[((a * 4 + bc) * N) * N + e];
    if (e < N) sL[a][e] = fl[(a * 4 + bc) * N + e];
  }
  for (int idx = tid; idx < 2 * ntc * ntc; idx += blockDim.x) sTM[idx / (ntc * ntc)][idx % (ntc * ntc)] = ftm[idx];
  const T rho = frho[cell];
  // stage r on the cell's nodes (Dirichlet nodes read as zero)
  constexpr int p = N - 1;
  for (int idx = tid; idx < n_t * NS; idx += blockDim.x) {
    const int j = idx / NS, a = idx % NS;
    const int lx = a % N, ly = (a / N) % N, lz = DIM == 3 ? a / (N * N) : 0;
    const int gx = cc[0] * p + lx, gy = cc[1] * p + ly, gz = cc[2] * p + lz;
    const bool in = gx != 0 && gx != g.nn[0] - 1 && gy != 0 && gy != g.nn[1] - 1 &&
                    (DIM == 2 || (gz != 0 && gz != g.nn[2] - 1));
    X[idx] = in ? r[(long long)j * g.nx + ((long long)gz * g.nn[1] + gy) * g.nn[0] + gx] : (T)0;
  }
  __syncthreads();
  // one 1D transform along axis `ax` of every line: forward (Q^T) or backward (Q)
  auto sweep = [&](int ax, bool forward) {
    constexpr int LINES = NS / N;
    const int stride = ax == 0 ? 1 : (ax == 1 ? N : N * N);
    for (int line = tid; line < n_t * LINES; line += blockDim.x) {
      const int j = line / LINES, l = line % LINES;
      int base;
      if (ax == 0) base = l * N;
      else if (ax == 1) base = (l % N) + (l / N) * N * N;
      else base = l;
      T* v = X + j * NS + base;
      T in[N], out[N];
#pragma unroll
      for (int k = 0; k < N; ++k) in[k] = v[k * stride];
#pragma unroll
      for (int i = 0; i < N; ++i) {
        T acc = 0;
#pragma unroll
        for (int k = 0; k < N; ++k) acc += (forward ? sQ[ax][k][i] : sQ[ax][i][k]) * in[k];
        out[i] = acc;
      }
#pragma unroll
      for (int i = 0; i < N; ++i) v[i * stride] = out[i];
    }
    __syncthreads();
  };
  for (int ax = 0; ax < DIM; ++ax) sweep(ax, true);
  // per mode s and time cell m: (rho lambda_s M_tau + N~) w = W[m, :, s]
  const int c = n_t / ntc;
  for (int pair = tid; pair < c * NS; pair += blockDim.x) {
    const int m = pair / NS, s = pair % NS;
    const int ix = s % N, iy = (s / N) % N, iz = DIM == 3 ? s / (N * N) : 0;
    const T lam = rho * (sL[0][ix] + sL[1][iy] + (DIM == 3 ? sL[2][iz] : (T)0));
    T A[FDM_MAXTC][FDM_MAXTC], b[FDM_MAXTC];
    for (int i = 0; i < ntc; ++i) {
      b[i] = X[(m * ntc + i) * NS + s];
      for (int k = 0; k < ntc; ++k) A[i][k] = lam * sTM[0][i * ntc + k] + sTM[1][i * ntc + k];
    }
    // Gaussian elimination with partial pivoting
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
  // add omega Z to the interior nodes (or to this cell's slot of the buffer)
  for (int idx = tid; idx < n_t * NS; idx += blockDim.x) {
    const int j = idx / NS, a = idx % NS;
    const int lx = a % N, ly = (a / N) % N, lz = DIM == 3 ? a / (N * N) : 0;
    if (cellbuf) {
      cellbuf[ebuf_index(g, j, cc[0], cc[1], cc[2], lx, ly, lz)] = omega * X[idx];
      continue;
    }
    const int gx = cc[0] * p + lx, gy = cc[1] * p + ly, gz = cc[2] * p + lz;
    const bool in = gx != 0 && gx != g.nn[0] - 1 && gy != 0 && gy != g.nn[1] - 1 &&
                    (DIM == 2 || (gz != 0 && gz != g.nn[2] - 1));
    if (in) u[(long long)j * g.nx + ((long long)gz * g.nn[1] + gy) * g.nn[0] + gx] += omega * X[idx];
  }
}

template <class T, int DIM, int N>
void launch_fdm(const GeomDesc& g, const ColourSet& cs, int n_t, int ntc, const T* fq, const T* fl,
                const T* frho, const T* ftm, const T* r, T* u, T omega, hipStream_t s, T* cb) {
  constexpr int NS = DIM == 3 ? N * N * N : N * N;
  const int nb = (int)cs.count;
  hipLaunchKernelGGL((k_asm_fdm<T, DIM, N>), dim3(nb), dim3(256), sizeof(T) * (size_t)n_t * NS, s, g, cs, n_t,
                     ntc, fq, fl, frho, ftm, r, u, omega, nb, cb);
}

}  // namespace

template <class T>
void asm_apply_fdm(const GeomDesc& g, int n_t, int nt_cell, const T* fq, const T* fl, const T* frho,
                   const T* ftm, const T* r, T* u, T omega, hipStream_t s, T* cellbuf, bool u_zero) {
  if (u_zero && !cellbuf) fail(STMG_E_ARG, "u_zero needs the per-cell buffer");
  if (nt_cell > FDM_MAXTC) fail(STMG_E_UNSUPPORTED, "too many temporal DoFs per time cell for the separable smoother");
  if ((size_t)n_t * (g.dim == 3 ? g.n * g.n * g.n : g.n * g.n) * sizeof(T) > 64 * 1024)
    fail(STMG_E_UNSUPPORTED, "cell too large for the separable smoother");
  const int nsets = cellbuf ? 1 : n_colours(g.dim);
  for (int colour = 0; colour < nsets; ++colour) {
    ColourSet cs = cellbuf ? all_cells(g) : colour_set(g, colour);
    if (cs.count == 0) continue;
    if (g.dim == 3) {
      switch (g.n) {
        case 2: launch_fdm<T, 3, 2>(g, cs, n_t, nt_cell, fq, fl, frho, ftm, r, u, omega, s, cellbuf); break;
        case 3: launch_fdm<T, 3, 3>(g, cs, n_t, nt_cell, fq, fl, frho, ftm, r, u, omega, s, cellbuf); break;
        case 4: launch_fdm<T, 3, 4>(g, cs, n_t, nt_cell, fq, fl, frho, ftm, r, u, omega, s, cellbuf); break;
        default: launch_fdm<T, 3, 5>(g, cs, n_t, nt_cell, fq, fl, frho, ftm, r, u, omega, s, cellbuf); break;
      }
    } else {
      switch (g.n) {
        case 2: launch_fdm<T, 2, 2>(g, cs, n_t, nt_cell, fq, fl, frho, ftm, r, u, omega, s, cellbuf); break;
        case 3: launch_fdm<T, 2, 3>(g, cs, n_t, nt_cell, fq, fl, frho, ftm, r, u, omega, s, cellbuf); break;
        case 4: launch_fdm<T, 2, 4>(g, cs, n_t, nt_cell, fq, fl, frho, ftm, r, u, omega, s, cellbuf); break;
        default: launch_fdm<T, 2, 5>(g, cs, n_t, nt_cell, fq, fl, frho, ftm, r, u, omega, s, cellbuf); break;
      }
    }
    STMG_CHECK_LAUNCH();
  }
  if (cellbuf) cell_gather<T>(g, n_t, cellbuf, u, s, nullptr, u_zero);
}

template void asm_apply_fdm<double>(const GeomDesc&, int, int, const double*, const double*, const double*,
                                    const double*, const double*, double*, double, hipStream_t, double*, bool);
template void asm_apply_fdm<float>(const GeomDesc&, int, int, const float*, const float*, const float*,
                                   const float*, const float*, float*, float, hipStream_t, float*, bool);

}  // namespace stmg
