// Host-callable launchers of the HIP kernels (all enqueue on the given stream).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "device.hpp"

namespace stmg {

// Host copy of the 1D tables of one spatial degree (row-major N x N).
struct LevelTables {
  int n = 0;
  std::vector<double> S, D, gq, gw;
};
LevelTables make_level_tables(int p);

// ---- operator (op_apply.hip) ----------------------------------------------------------
// y += scale * S_interior x : interior rows only, Dirichlet columns ignored.
// With cellbuf (ncells * n_t * (p+1)^d entries) every cell writes its contribution there in
// one launch and a node gather adds them to y (coarse levels: two launches instead of one
// per colour); without it the cells are processed colour by colour.
template <class T>
void st_apply(const GeomDesc& g, const LevelTables& lt, const TemporalDev<T>& tp, const T* x, T* y,
              T scale, hipStream_t s, T* cellbuf = nullptr, const T* base = nullptr, bool overwrite = false);
// Every level uses the per-cell buffer path: one launch over all cells plus a gather beats 2^d
// colour launches with read-modify-write in both precisions.  Levels with at most this many cells
// always allocate the buffer; larger levels allocate it best-effort and run on the colour path
// when device memory is short.
constexpr long long TWO_PHASE_MAX_CELLS = 4096;
// Gather of the per-cell buffer (fixed cell order) into the lattice vector.
// y += sum of the cell contributions (overwrite = false), or y = base + sum (overwrite = true,
// base may be null for zero; Dirichlet nodes then receive base, or zero)
template <class T> void cell_gather(const GeomDesc& g, int n_t, const T* cb, T* y, hipStream_t s,
                                    const T* base = nullptr, bool overwrite = false);

// ---- brick operator (op_brick.hip) -----------------------------------------------------------
// 1D reference mass and stiffness of Q_p on [0, 1] (GLL nodal basis, exact Gauss quadrature),
// row-major n x n.  Host only.
struct CartTables {
  int n = 0;
  std::vector<double> M, K;
};
CartTables make_cart_tables(const LevelTables& lt);
// 3D level with axis-aligned box cells and one coefficient per cell
bool brick_applicable(const GeomDesc& g);
// y = base + scale * S_interior x on interior rows (overwrite; base null: zero; Dirichlet rows of y
// receive base or zero) or y += scale * S_interior x; bricks of cells staged in LDS, 2^3 brick
// colours, no per-cell buffer.
template <class T>
void st_apply_brick(const GeomDesc& g, const CartTables& ct, const TemporalDev<T>& tp, const T* x, T* y,
                    T scale, hipStream_t s, const T* base, bool overwrite);

// ---- vector kernels (blas.hip) --------------------------------------------------------------
template <class T> void fill(T* y, T v, long long n, hipStream_t s);
template <class T> void copy(const T* x, T* y, long long n, hipStream_t s);
template <class T> void axpy(T a, const T* x, T* y, long long n, hipStream_t s);          // y += a x
template <class T> void axpby(T a, const T* x, T b, T* y, long long n, hipStream_t s);    // y = a x + b y
template <class T> void scal(T a, T* y, long long n, hipStream_t s);
void cast_d2f(const double* x, float* y, long long n, hipStream_t s);
void cast_f2d(const float* x, double* y, long long n, hipStream_t s);
// On Dirichlet nodes (list bidx of length nb, per temporal plane of nx nodes, n_t planes):
// y[b] = a * x[b] + c * y[b].
template <class T>
void boundary_axpby(const int* bidx, long long nb, long long nx, int n_t, T a, const T* x, T c, T* y,
                    hipStream_t s);
// Reduction workspace: RED_BLOCKS * PS doubles of device memory (JC vectors per pass plus one).
constexpr int RED_BLOCKS = 1024;
constexpr int JC = 32;
constexpr int PS = JC + 1;
// out[j] = sum_i V_j[i] * w[i] for j < k (V_j = V + j * ldv), double accumulation; out on device.
// With self = true also out[k] = w . w.  Vectors are read once per group of JC.
void multi_dot(const double* V, long long ldv, int k, const double* w, long long n, double* out,
               double* ws, hipStream_t s, bool self = false);
// w -= sum_j h[j] V_j  (h on device)
void multi_axpy_neg(const double* V, long long ldv, int k, const double* h, double* w, long long n,
                    hipStream_t s);
// w -= sum_j h[j] hs[j] V_j (hs on device, null: 1), then out[0] = w . w and out[1] = 1 if w holds
// NaN/Inf (else 0)
void multi_axpy_neg_norm(const double* V, long long ldv, int k, const double* h, double* w, long long n,
                         double* out, double* ws, hipStream_t s, const double* hs = nullptr);
// x += sum_j y[j] Z_j  (y on device, Z in T)
template <class T>
void multi_axpy_acc(const T* Z, long long ldz, int k, const double* y, double* x, long long n,
                    hipStream_t s);
// out[0] = sum x^2 (double accumulation), out[1] = 1 if a non-finite value was seen
template <class T> void norm2_check(const T* x, long long n, double* out, double* ws, hipStream_t s);

// ---- transfers (transfer.hip) ---------------------------------------------------------------
// One 1D sweep along axis `ax` of a [n_t][n2][n1][n0] array (x fastest):
// out[.., i, ..] (+)= sum_{k in row i} w[k] * in[.., col[k], ..] with CSR (ptr, col, w).
template <class T>
void sweep1d(const T* in, T* out, int n_t, const int in_dims[3], int ax, int out_len, const int* ptr,
             const int* col, const T* w, int nnz, int max_row, bool accumulate, hipStream_t s);

// Fused 3D tensor-product transfer (transfer.hip): out (+)= (Az (x) Ay (x) Ax) in on each of n_t
// planes, with banded 1D factors.  Outputs are tiled in T[0] x T[1] boxes in x and y (T[0] a power
// of two, T[0] T[1] <= 256) and chunks of T[2] (16 or 4) planes in z.  Tables per axis (T3Axis):
// for every tile (x, y) or chunk (z) the first and last input index it reads (lo > hi: all its rows
// are empty); for x and y every output row's kmax (column - lo of the row's tile, weight) pairs,
// padded with zero weights and column 0; for z the chunk's dense weights [chunk][T[2]][S[2]].  S is
// the largest input span of a tile per axis (S[0] S[1] <= 2048).  ok is false when no tile fits or
// an x or y row is longer than the kernel's largest kmax; then the transfer runs as 1D sweeps.
struct Tensor3Plan {
  int T[3] = {1, 1, 1};
  int lg[3] = {0, 0, 0};
  int S[3] = {1, 1, 1};
  int nt[3] = {1, 1, 1};
  int kmax = 2;
  bool ok = false;
};
struct T3Axis {
  const int* lo;      // [tiles]
  const int* hi;      // [tiles]
  const int* col;     // x, y: [rows][kmax]; z: unused
  const void* w;      // x, y: [rows][kmax]; z: [chunks][T[2]][S[2]]; element type T
};
template <class T>
void tensor3(const T* in, T* out, int n_t, const int in_dims[3], const int out_dims[3], const Tensor3Plan& pl,
             const T3Axis ax[3], bool accumulate, hipStream_t s);

// Temporal transfer on the interior nodes of one spatial lattice of nx nodes (transfer.hip):
// mode 0: out = (P (x) I) in, 1: out += (P (x) I) in, 2: out = (P^T (x) I) in, with P the dense
// (nf x nc) temporal prolongation; vectors are [plane][node], Dirichlet nodes give zero.
constexpr int TT_MAX = 32;
template <class T>
void time_transfer(const T* P, int nf, int nc, long long nx, const unsigned char* mask, const T* in, T* out,
                   int mode, hipStream_t s);

// ---- smoother (asm.hip) ----------------------------------------------------------------------
// Set-up: probe vectors (two planes) for colour `colour` (of 3^dim) and cell-local node b.
void asm_probe_set(const GeomDesc& g, int colour, int b, double val, double* x, hipStream_t s);
// Column b of A_KK (plane 0 of y) and M_KK (plane 1) for every cell of the colour;
// blocks are column-major n_s x n_s per cell; Dirichlet nodes become identity rows/columns.
void asm_extract(const GeomDesc& g, int colour, int b, const double* y, double* Ablk, double* Mblk,
                 hipStream_t s);
// Tinv[K][s] = (lam[K][s] M_tau + N~)^{-1} (nt x nt, row-major); *bad set if singular.
template <class T>
void asm_tinv(long long ncells, int ns, int nt, const double* lam, const double* Mtau, const double* Nt,
              T* Tinv, int* bad, hipStream_t s);
template <class Tout> void convert_from_double(const double* a, Tout* b, long long n, hipStream_t s);
// u += omega * sum_K R_K^T (I (x) Q_K) Tinv_K (I (x) Q_K^T) R_K r on interior rows.
// cellbuf: as for st_apply (per-cell corrections, then a node gather).  u_zero (only with
// cellbuf): u is taken as zero on entry and not read; the gather writes every node of u.
template <class T>
void asm_apply(const GeomDesc& g, int n_t, int nt_cell, const T* Q, const T* Tinv, const T* r, T* u,
               T omega, hipStream_t s, T* cellbuf = nullptr, bool u_zero = false);

// Separable (fast diagonalisation) variant on Cartesian levels:
//   u += omega * sum_K R_K^T (I (x) Q) [rho_K lambda_s M_tau + N~]^{-1} (I (x) Q^T) R_K r,
// Q = Q_z (x) Q_y (x) Q_x from per-axis 1D generalised eigenproblems (tables fq [3][4][n][n],
// fl [3][4][n] by axis and boundary case), frho per cell, ftm = [M_tau; N~] (nt_cell^2 each).
template <class T>
void asm_apply_fdm(const GeomDesc& g, int n_t, int nt_cell, const T* fq, const T* fl, const T* frho,
                   const T* ftm, const T* r, T* u, T omega, hipStream_t s, T* cellbuf = nullptr,
                   bool u_zero = false);

// Brick-tiled separable smoother (asm_brick.hip) on 3D Cartesian levels with one or two temporal
// DoFs per time cell: same result as asm_apply_fdm; Mtau, Ntil are the host (nt_cell x nt_cell,
// row-major) time-cell matrices; u_zero: u is zero on entry and not read.
bool fdm_brick_applicable(const GeomDesc& g, int nt_cell);
template <class T>
void asm_apply_fdm_brick(const GeomDesc& g, int n_t, int nt_cell, const double* Mtau, const double* Ntil,
                         const T* fq, const T* fl, const T* frho, const T* r, T* u, T omega, bool u_zero,
                         hipStream_t s);

// Separable vertex-patch smoother (asm_patch.hip): u += omega * sum over interior vertices v and
// time cells of the patch block solve (2p - 1 inner nodes per axis); pq: per axis the 1D
// eigenvectors (P x P, row-major, Q(r, c) at r P + c), pl: their eigenvalues (P per axis), prho: the
// mean coefficient per interior vertex ((nc_x - 1)(nc_y - 1)(nc_z - 1), x fastest), ptm: M_tau then
// N~ (nt_cell x nt_cell each).  patch_applicable: Cartesian, at least two cells per direction.
bool patch_applicable(const GeomDesc& g, int nt_cell);
template <class T>
void asm_apply_patch(const GeomDesc& g, int n_t, int nt_cell, const T* pq, const T* pl, const T* prho, const T* ptm,
                     const T* r, T* u, T omega, hipStream_t s);

// ---- smoother set-up check (hierarchy.hip) ----------------------------------------------------
// flag[c] = 1 unless cell c's eigenpairs pass: max|R - I| <= tol for R = Q^T M Q, and per column k
// max|AQ(:, k) - lambda_k T(:, k)| <= tol (max|AQ(:, k)| + |lambda_k| max|T(:, k)|) for T = M Q
// (column-major ns x ns blocks, ncells <= 2^31 - 1).
void asm_eig_check(long long ncells, int ns, const double* R, const double* AQ, const double* T,
                   const double* lam, double tol, int* flag, hipStream_t s);

// ---- coarse solve (coarse.hip) ---------------------------------------------------------------------
// z[idx[i]] = sum_j Cinv[i][j] f[idx[j]] for the m interior DoFs of the coarsest level.
template <class T>
void coarse_apply(const T* Cinv, const long long* idx, int m, const T* f, T* z, hipStream_t s);

}  // namespace stmg
