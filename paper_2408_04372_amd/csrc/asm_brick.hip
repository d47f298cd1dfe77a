// Brick-tiled separable (fast diagonalisation) variant of the space-time cell-wise additive
// Schwarz smoother (Section 3.3, eqs. vanka0, vanka):
//   u += omega * sum_{K, m} R_{K,m}^T (I (x) Q) [rho_K Lambda (x) M_tau + I (x) N~]^{-1} (I (x) Q^T) R_{K,m} r
// with Q = Q_z (x) Q_y (x) Q_x from the per-axis 1D generalised eigenproblems of the cell's 1D mass
// and stiffness (tables by axis and boundary case, as for k_asm_fdm) and Lambda the sums of the 1D
// eigenvalues; one ntc x ntc temporal solve per spatial mode and time cell.
//
// MI355X mapping (brick tiling in brick.hpp).  A team of ntc (p+1) lanes owns one (cell, time
// cell); lane (d, t) (team lane NTC t + d) holds temporal DoF d and first the y = t plane ([z][x]:
// the forward x and z transforms are lane local); a per-x-slice exchange through a small LDS scratch
// hands it the z = t plane ([y][x]), where it applies Q_y^T, the temporal solves of its modes (the
// other temporal DoF of a mode comes from the neighbouring lane by a DPP permutation) and Q_y,
// then Q_x; a second per-slice exchange returns the y = t plane, where Q_z completes the correction.  The 1D tables sit in LDS; the corrections are summed into
// the brick's LDS copy by cell parity class and written once per node.
#include "brick.hpp"

namespace stmg {

namespace {

template <class T, int NTC>
struct BrickFdmArgs {
  T Mt[NTC][NTC];     // M_tau of one time cell
  T Nt[NTC][NTC];     // N~ of one time cell
  GeomDesc g;
  const T* fq;        // [3][4][N][N] eigenvectors (columns) by axis and boundary case
  const T* fl;        // [3][4][N] eigenvalues
  const T* frho;      // cell-mean coefficient per cell
  const T* r;
  T* u;
  T omega;
  int overwrite;      // u is zero on entry and not read
  int n_t;            // c * NTC temporal planes
  BrickLaunch L;
};

// 1 / a: the hardware estimate refined by two Newton-Raphson steps r <- r + r (1 - a r) (FP64), or
// the division (FP32)
__device__ inline double recip(double a) {
  double r = __builtin_amdgcn_rcp(a);
  r = fma(fma(-a, r, 1.0), r, r);
  r = fma(fma(-a, r, 1.0), r, r);
  return r;
}
__device__ inline float recip(float a) { return 1.0f / a; }

// the value of lane l ^ 1 (DPP quad permutation [1, 0, 3, 2]; every lane of the wave is active)
__device__ inline float pair_swap(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ inline double pair_swap(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// In-place 1D transform of the lane's 5 x 5 plane A[r][c] along the column index (ALONG_COL) or the
// row index, with the N x N table Qt in LDS: forward out_i = sum_k Q(k, i) in_k, backward
// out_i = sum_k Q(i, k) in_k.  The table is read once per call into registers.
template <class T, int N, bool ALONG_COL, bool FORWARD>
__device__ inline void sweep_inplace(const T* Qt, T (&A)[N][N]) {
  T q[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int k = 0; k < N; ++k) q[i][k] = FORWARD ? Qt[k * N + i] : Qt[i * N + k];
#pragma unroll
  for (int l = 0; l < N; ++l) {
    T in[N];
#pragma unroll
    for (int k = 0; k < N; ++k) in[k] = ALONG_COL ? A[l][k] : A[k][l];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T acc = 0;
#pragma unroll
      for (int k = 0; k < N; ++k) acc += q[i][k] * in[k];
      if (ALONG_COL) A[l][i] = acc;
      else A[i][l] = acc;
    }
  }
}

template <class T, int N, int NTC>
__global__ __launch_bounds__(512) void k_asm_fdm_brick(BrickFdmArgs<T, NTC> A) {
  constexpr int p = N - 1;
  constexpr int TL = NTC * N;                         // lanes per team: (temporal DoF d, plane t)
  constexpr int TPW = 64 / TL;
  constexpr int NN = N * N;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const GeomDesc& g = A.g;
  const int n_t = A.n_t, c = n_t / NTC;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int nbx = A.L.NBd[0], nby = A.L.NBd[1];
  const BrickPos P = brick_pos(A.L, g);
  const int NB = P.NB;
  const int teams = (nthr >> 6) * TPW;
  T* xs = reinterpret_cast<T*>(smem_raw);            // [n_t][NB]: r, then the brick's corrections
  T* scr = xs + (size_t)n_t * NB;                     // [teams][NTC][N][N] exchange slices
  T* sQ = scr + (size_t)teams * NTC * NN;             // [3][4][N][N]
  T* sL = sQ + 3 * 4 * NN;                            // [3][4][N]
  T* zl = sL + 3 * 4 * N;                             // one zero
  for (int e = tid; e < 3 * 4 * NN; e += nthr) sQ[e] = A.fq[e];
  for (int e = tid; e < 3 * 4 * N; e += nthr) sL[e] = A.fl[e];
  if (tid == 0) *zl = (T)0;
  brick_stage<T, 24>(g, A.L, P, n_t, A.r, xs);
  __syncthreads();

  const int wave = tid >> 6, lane = tid & 63;
  const int tw = lane / TL, tl = lane - tw * TL;
  const int d = tl % NTC, t = tl / NTC;               // this lane's temporal DoF and plane
  const int team = wave * TPW + tw;
  const int ncell = P.nc[0] * P.nc[1] * P.nc[2];
  const bool act = tw < TPW && team < ncell * c;
  const int lc = act ? team / c : 0, m = act ? team - lc * c : 0;
  const int lcx = lc % P.nc[0], lcy = (lc / P.nc[0]) % P.nc[1], lcz = lc / (P.nc[0] * P.nc[1]);
  const int cc[3] = {P.c0[0] + lcx, P.c0[1] + lcy, P.c0[2] + lcz};
  const long long cell = ((long long)cc[2] * g.nc[1] + cc[1]) * g.nc[0] + cc[0];
  const T rho = act ? A.frho[cell] : (T)1;
  const T* Q[3];
  const T* lam[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int bc = (cc[a] == 0 ? 1 : 0) + (cc[a] == g.nc[a] - 1 ? 2 : 0);
    Q[a] = sQ + (a * 4 + bc) * NN;
    lam[a] = sL + (a * 4 + bc) * N;
  }
  // lane (d, t = y): R[z][x] of plane m NTC + d (Dirichlet nodes are zero in xs)
  T R[N][N];
  {
    const T* xc = xs + (size_t)(m * NTC + d) * NB + ((size_t)(lcz * p) * nby + (lcy * p + t)) * nbx + lcx * p;
#pragma unroll
    for (int z = 0; z < N; ++z)
#pragma unroll
      for (int x = 0; x < N; ++x) R[z][x] = xc[z * nby * nbx + x];
  }
  __syncthreads();                                    // every team has read its input
  for (int e = tid; e < n_t * NB; e += nthr) xs[e] = (T)0;
  __syncthreads();

  // forward transforms along x and z (lane local)
  sweep_inplace<T, N, true, true>(Q[0], R);          // R[z][x]: along x
  sweep_inplace<T, N, false, true>(Q[2], R);         // along z

  // exchange 1, one x slice at a time: lane (d, t = z) receives the y column ([y][x])
  T S[N][N];
  T* sc = scr + (size_t)(act ? team : 0) * NTC * NN + d * NN;
#pragma unroll
  for (int xx = 0; xx < N; ++xx) {
    if (act) {
#pragma unroll
      for (int z = 0; z < N; ++z) sc[z * N + t] = R[z][xx];
    }
    wave_sync_lds();
#pragma unroll
    for (int y = 0; y < N; ++y) S[y][xx] = act ? sc[t * N + y] : (T)0;
    wave_sync_lds();
  }
  sweep_inplace<T, N, false, true>(Q[1], S);         // S[y][x]: along y
  // temporal solve (lam M_tau + N~) w = b of every mode (x, y, z = t), lam = rho (lx + ly + lz), in
  // closed form (Cramer's rule for two temporal DoFs); with two, the mode's other DoF sits in the
  // neighbouring lane (lane = team base + NTC t + d) and each lane forms its own component
  {
    const T lz_t = lam[2][t];
    T lx[N], ly[N];
#pragma unroll
    for (int k = 0; k < N; ++k) { lx[k] = lam[0][k]; ly[k] = lam[1][k]; }
#pragma unroll
    for (int y = 0; y < N; ++y)
#pragma unroll
      for (int x = 0; x < N; ++x) {
        const T lm = rho * (lx[x] + ly[y] + lz_t);
        if constexpr (NTC == 1) {
          S[y][x] = S[y][x] * recip(lm * A.Mt[0][0] + A.Nt[0][0]);
        } else {
          const T own = S[y][x], oth = pair_swap(own);
          const T a00 = lm * A.Mt[0][0] + A.Nt[0][0], a01 = lm * A.Mt[0][1] + A.Nt[0][1];
          const T a10 = lm * A.Mt[1][0] + A.Nt[1][0], a11 = lm * A.Mt[1][1] + A.Nt[1][1];
          const T inv = recip(a00 * a11 - a01 * a10);
          S[y][x] = (d == 0 ? a11 * own - a01 * oth : a00 * own - a10 * oth) * inv;
        }
      }
  }
  sweep_inplace<T, N, false, false>(Q[1], S);        // back along y
  sweep_inplace<T, N, true, false>(Q[0], S);         // back along x

  // exchange 2, one x slice at a time: lane (d, t = y) receives the z column ([z][x])
  T O[N][N];
#pragma unroll
  for (int xx = 0; xx < N; ++xx) {
    if (act) {
#pragma unroll
      for (int y = 0; y < N; ++y) sc[t * N + y] = S[y][xx];
    }
    wave_sync_lds();
#pragma unroll
    for (int z = 0; z < N; ++z) O[z][xx] = act ? sc[z * N + t] : (T)0;
    wave_sync_lds();
  }
  sweep_inplace<T, N, false, false>(Q[2], O);        // back along z

  // sum the corrections into the brick, one cell parity class per round (cells of a class share no
  // node, so each sum meets no other one and the order is fixed)
  const int par = (lcx & 1) | ((lcy & 1) << 1) | ((lcz & 1) << 2);
  T* o = xs + (size_t)(m * NTC + d) * NB + ((size_t)(lcz * p) * nby + (lcy * p + t)) * nbx + lcx * p;
  for (int rr = 0; rr < 8; ++rr) {
    if (act && par == rr) {
#pragma unroll
      for (int z = 0; z < N; ++z)
#pragma unroll
        for (int x = 0; x < N; ++x) {
          if constexpr (sizeof(T) == 8)    // one LDS add instruction (measured slower for FP32)
            __hip_atomic_fetch_add(o + z * nby * nbx + x, O[z][x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          else
            o[z * nby * nbx + x] += O[z][x];
        }
    }
    __syncthreads();
  }

  brick_write<T, 24>(g, A.L, P, n_t, xs, zl, A.omega, A.overwrite, (const T*)nullptr, A.u);
}

template <class T, int N, int NTC>
void launch_fdm_brick(const GeomDesc& g, int n_t, const double* Mtau, const double* Ntil, const T* fq,
                      const T* fl, const T* frho, const T* r, T* u, T omega, bool u_zero, hipStream_t s) {
  BrickFdmArgs<T, NTC> A;
  for (int i = 0; i < NTC; ++i)
    for (int k = 0; k < NTC; ++k) {
      A.Mt[i][k] = (T)Mtau[i * NTC + k];
      A.Nt[i][k] = (T)Ntil[i * NTC + k];
    }
  A.g = g;
  A.fq = fq;
  A.fl = fl;
  A.frho = frho;
  A.r = r;
  A.u = u;
  A.omega = omega;
  A.overwrite = u_zero ? 1 : 0;
  A.n_t = n_t;
  BrickPlan pl;
  static const int vgprs = kernel_vgprs(k_asm_fdm_brick<T, N, NTC>);
  if (!plan_brick(g, n_t, n_t / NTC, NTC * N, sizeof(T), NTC * N * N, sizeof(T) * (3 * 4 * (N * N + N) + 1), vgprs, pl))
    fail(STMG_E_UNSUPPORTED, "no brick fits the temporal DoFs of the smoother");
  BrickLaunch L[8];
  brick_launches(g, pl, L);
  for (int colour = 0; colour < 8; ++colour) {
    if (L[colour].nblocks == 0) continue;
    A.L = L[colour];
    hipLaunchKernelGGL((k_asm_fdm_brick<T, N, NTC>), dim3((unsigned)L[colour].nblocks), dim3(pl.waves * 64),
                       pl.lds, s, A);
    STMG_CHECK_LAUNCH();
  }
}

template <class T, int N>
void fdm_brick_ntc(const GeomDesc& g, int n_t, int ntc, const double* Mtau, const double* Ntil, const T* fq,
                   const T* fl, const T* frho, const T* r, T* u, T omega, bool u_zero, hipStream_t s) {
  switch (ntc) {
    case 1: launch_fdm_brick<T, N, 1>(g, n_t, Mtau, Ntil, fq, fl, frho, r, u, omega, u_zero, s); break;
    case 2: launch_fdm_brick<T, N, 2>(g, n_t, Mtau, Ntil, fq, fl, frho, r, u, omega, u_zero, s); break;
    default: fail(STMG_E_UNSUPPORTED, "brick smoother: 1 or 2 temporal DoFs per time cell");
  }
}

}  // namespace

// the smoother takes one coefficient per cell (frho), so levels with quadrature-point coefficients
// qualify as well
bool fdm_brick_applicable(const GeomDesc& g, int nt_cell) {
  return g.dim == 3 && !g.verts && g.n >= 2 && g.n <= MAXN && nt_cell >= 1 && nt_cell <= 2;
}

template <class T>
void asm_apply_fdm_brick(const GeomDesc& g, int n_t, int nt_cell, const double* Mtau, const double* Ntil,
                         const T* fq, const T* fl, const T* frho, const T* r, T* u, T omega, bool u_zero,
                         hipStream_t s) {
  if (!fdm_brick_applicable(g, nt_cell)) fail(STMG_E_UNSUPPORTED, "the brick smoother needs a 3D Cartesian level");
  if (g.ncells == 0 || n_t == 0) return;
  if (n_t % nt_cell) fail(STMG_E_ARG, "temporal planes are not whole time cells");
  switch (g.n) {
    case 2: fdm_brick_ntc<T, 2>(g, n_t, nt_cell, Mtau, Ntil, fq, fl, frho, r, u, omega, u_zero, s); break;
    case 3: fdm_brick_ntc<T, 3>(g, n_t, nt_cell, Mtau, Ntil, fq, fl, frho, r, u, omega, u_zero, s); break;
    case 4: fdm_brick_ntc<T, 4>(g, n_t, nt_cell, Mtau, Ntil, fq, fl, frho, r, u, omega, u_zero, s); break;
    case 5: fdm_brick_ntc<T, 5>(g, n_t, nt_cell, Mtau, Ntil, fq, fl, frho, r, u, omega, u_zero, s); break;
    default: fail(STMG_E_UNSUPPORTED, "p must be 1..4");
  }
}

template void asm_apply_fdm_brick<double>(const GeomDesc&, int, int, const double*, const double*, const double*,
                                          const double*, const double*, const double*, double*, double, bool,
                                          hipStream_t);
template void asm_apply_fdm_brick<float>(const GeomDesc&, int, int, const double*, const double*, const float*,
                                         const float*, const float*, const float*, float*, float, bool, hipStream_t);

}  // namespace stmg
