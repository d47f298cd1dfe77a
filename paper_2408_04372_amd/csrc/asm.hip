// Space-time cell-wise additive Schwarz smoother (Section 3.3, eqs. vanka0, vanka).
//
// The block of space-time cell K x I_m is the principal submatrix of the level
// operator on K's interior nodes and I_m's temporal DoFs.  Because the slab
// operator is M_T (x) A_h + N_T (x) M_h, that block is
//     B_K = M_tau (x) A_KK + N~ (x) M_KK,
// the same for every time cell m (M_tau, N~: diagonal blocks of M_T, N_T), with
// A_KK, M_KK the principal submatrices of the assembled spatial matrices.  The
// paper only uses this structure to avoid assembling S; here it also factorises
// the local solve: with the generalised eigenpairs A_KK Q = M_KK Q Lambda,
// Q^T M_KK Q = I,
//     B_K^{-1} = (I (x) Q) blockdiag_s (lambda_s M_tau + N~)^{-1} (I (x) Q^T),
// so one application per spatial cell is two dense [n_s x n_s] x [n_s x n_t]
// products (all time cells of the slab at once) and n_s tiny N_t x N_t solves,
// instead of a dense (N_t n_s)^2 inverse per block.  Corrections are written to a
// per-cell buffer and summed by a node gather, or, without a buffer, blocks are
// applied in 2^d colours of cells that share no node; neither uses atomics.
// Dirichlet nodes inside a
// block are decoupled (identity rows in A_KK and M_KK) and masked on input and
// output, so they never receive a correction from the block.
//
// Set-up kernels: probe vectors for extracting A_KK / M_KK from the matrix-free
// operator (3^d colours of cells whose node sets are far enough apart), the
// extraction itself, and the per-mode temporal inverses.
#include "kernels.hpp"

namespace stmg {

namespace {

__device__ inline void cell_coords(long long cell, const GeomDesc& g, int& cx, int& cy, int& cz) {
  cx = (int)(cell % g.nc[0]);
  cy = (int)((cell / g.nc[0]) % g.nc[1]);
  cz = (int)(cell / ((long long)g.nc[0] * g.nc[1]));
}

// node index and interior flag of local node r = lx + n (ly + n lz) of a cell
__device__ inline long long node_of(const GeomDesc& g, int cx, int cy, int cz, int r, bool& interior) {
  int n = g.n, p = g.p;
  int lx = r % n, ly = (r / n) % n, lz = (g.dim == 3) ? r / (n * n) : 0;
  int gx = cx * p + lx, gy = cy * p + ly, gz = cz * p + lz;
  interior = gx != 0 && gx != g.nn[0] - 1 && gy != 0 && gy != g.nn[1] - 1 &&
             (g.dim == 2 || (gz != 0 && gz != g.nn[2] - 1));
  return ((long long)gz * g.nn[1] + gy) * g.nn[0] + gx;
}

__device__ inline bool in_colour(const GeomDesc& g, int cx, int cy, int cz, int colour) {
  int ox = colour % 3, oy = (colour / 3) % 3, oz = colour / 9;
  return (cx % 3) == ox && (cy % 3) == oy && (g.dim == 2 || (cz % 3) == oz);
}

// x[plane t][node(K, b)] = val for every cell K of the colour, both planes
__global__ void k_probe_set(GeomDesc g, int colour, int b, double val, double* x) {
  for (long long cell = blockIdx.x * (long long)blockDim.x + threadIdx.x; cell < g.ncells;
       cell += (long long)gridDim.x * blockDim.x) {
    int cx, cy, cz;
    cell_coords(cell, g, cx, cy, cz);
    if (!in_colour(g, cx, cy, cz, colour)) continue;
    bool in;
    long long node = node_of(g, cx, cy, cz, b, in);
    x[node] = val;
    x[g.nx + node] = val;
  }
}

// column b of the principal blocks of every cell of the colour (column-major n_s x n_s)
__global__ void k_extract(GeomDesc g, int colour, int b, const double* y, double* Ablk, double* Mblk) {
  const int ns = (g.dim == 3) ? g.n * g.n * g.n : g.n * g.n;
  long long total = g.ncells * ns;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    long long cell = idx / ns;
    int a = (int)(idx - cell * ns);
    int cx, cy, cz;
    cell_coords(cell, g, cx, cy, cz);
    if (!in_colour(g, cx, cy, cz, colour)) continue;
    bool ina, inb;
    long long na = node_of(g, cx, cy, cz, a, ina);
    (void)node_of(g, cx, cy, cz, b, inb);
    double av, mv;
    if (!ina || !inb) {
      av = mv = (a == b) ? 1.0 : 0.0;     // Dirichlet node: decoupled identity row/column
    } else {
      av = y[na];
      mv = y[g.nx + na];
    }
    size_t off = (size_t)cell * ns * ns + (size_t)b * ns + a;
    Ablk[off] = av;
    Mblk[off] = mv;
  }
}

// Tinv[K][s] = (lambda_{K,s} M_tau + N~)^{-1}, Gauss-Jordan with partial pivoting per thread
template <class T>
__global__ void k_tinv(long long ncells, int ns, int nt, const double* __restrict__ lam,
                       const double* __restrict__ Mtau, const double* __restrict__ Nt, T* Tinv,
                       int* bad) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < ncells * ns;
       idx += (long long)gridDim.x * blockDim.x) {
    double l = lam[idx];
    double A[6][12];
    for (int i = 0; i < nt; ++i)
      for (int j = 0; j < nt; ++j) {
        A[i][j] = l * Mtau[i * nt + j] + Nt[i * nt + j];
        A[i][nt + j] = (i == j) ? 1.0 : 0.0;
      }
    for (int c = 0; c < nt; ++c) {
      int pr = c;
      for (int r = c + 1; r < nt; ++r)
        if (fabs(A[r][c]) > fabs(A[pr][c])) pr = r;
      if (A[pr][c] == 0.0) { *bad = 1; break; }
      if (pr != c)
        for (int j = 0; j < 2 * nt; ++j) { double tmp = A[c][j]; A[c][j] = A[pr][j]; A[pr][j] = tmp; }
      double d = 1.0 / A[c][c];
      for (int j = 0; j < 2 * nt; ++j) A[c][j] *= d;
      for (int r = 0; r < nt; ++r) {
        if (r == c) continue;
        double f = A[r][c];
        for (int j = 0; j < 2 * nt; ++j) A[r][j] -= f * A[c][j];
      }
    }
    T* out = Tinv + idx * nt * nt;
    for (int i = 0; i < nt; ++i)
      for (int j = 0; j < nt; ++j) out[i * nt + j] = (T)A[i][nt + j];
  }
}

template <class Tin, class Tout>
__global__ void k_convert(const Tin* __restrict__ a, Tout* __restrict__ b, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    b[i] = (Tout)a[i];
}

constexpr int ABS = 256;   // threads per workgroup of the apply kernel
constexpr int JMAX = 32;   // accumulators per thread

// u += omega * sum_K R_K^T B_K^{-1} R_K r   (interior rows; one workgroup per spatial cell)
template <class T>
__global__ __launch_bounds__(ABS) void k_asm_apply(GeomDesc g, ColourSet cs, int n_t, int nt_cell,
                                                   const T* __restrict__ Q, const T* __restrict__ Tinv,
                                                   const T* __restrict__ r, T* __restrict__ u, T omega,
                                                   int nblocks, T* __restrict__ cellbuf) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ns = (g.dim == 3) ? g.n * g.n * g.n : g.n * g.n;
  T* R = reinterpret_cast<T*>(smem_raw);     // [n_t][ns]
  T* W = R + (size_t)n_t * ns;               // [n_t][ns]
  const long long li = xcd_swizzle(blockIdx.x, nblocks);
  if (li >= cs.count) return;
  int cx, cy, cz;
  const long long cell = colour_cell(cs, g, li, cx, cy, cz);
  const int tid = threadIdx.x;
  for (int idx = tid; idx < n_t * ns; idx += ABS) {
    int j = idx / ns, a = idx - j * ns;
    bool in;
    long long node = node_of(g, cx, cy, cz, a, in);
    R[idx] = in ? r[(long long)j * g.nx + node] : (T)0;
  }
  __syncthreads();
  const T* Qc = Q + (size_t)cell * ns * ns;     // column-major: Q(a, s) = Qc[s * ns + a]
  const int JG = ABS / ns > 0 ? ABS / ns : 1;  // j-groups
  const int o = tid % ns, jg = tid / ns;
  const bool on = jg < JG && tid < JG * ns;
  // W[j][s] = sum_a Q(a, s) R[j][a]   (this thread: s = o, j = jg + jj * JG)
  if (on) {
    T acc[JMAX];
#pragma unroll
    for (int jj = 0; jj < JMAX; ++jj) acc[jj] = 0;
    const T* qcol = Qc + (size_t)o * ns;
    for (int a = 0; a < ns; ++a) {
      T q = qcol[a];
#pragma unroll
      for (int jj = 0; jj < JMAX; ++jj) {
        int j = jg + jj * JG;
        if (j < n_t) acc[jj] += q * R[j * ns + a];
      }
    }
#pragma unroll
    for (int jj = 0; jj < JMAX; ++jj) {
      int j = jg + jj * JG;
      if (j < n_t) W[j * ns + o] = acc[jj];
    }
  }
  __syncthreads();
  // per mode s and time cell m: W[m, :, s] <- (lambda_s M_tau + N~)^{-1} W[m, :, s]
  const int c = n_t / nt_cell;
  for (int idx = tid; idx < c * ns; idx += ABS) {
    int m = idx / ns, s = idx - m * ns;
    const T* Ti = Tinv + ((size_t)cell * ns + s) * nt_cell * nt_cell;
    T w[8], v[8];
    for (int b = 0; b < nt_cell; ++b) w[b] = W[(m * nt_cell + b) * ns + s];
    for (int a = 0; a < nt_cell; ++a) {
      T acc = 0;
      for (int b = 0; b < nt_cell; ++b) acc += Ti[a * nt_cell + b] * w[b];
      v[a] = acc;
    }
    for (int a = 0; a < nt_cell; ++a) W[(m * nt_cell + a) * ns + s] = v[a];
  }
  __syncthreads();
  // Z[j][a] = sum_s Q(a, s) W[j][s]; scatter-add omega * Z to the interior nodes
  if (on) {
    T acc[JMAX];
#pragma unroll
    for (int jj = 0; jj < JMAX; ++jj) acc[jj] = 0;
    for (int s = 0; s < ns; ++s) {
      T q = Qc[(size_t)s * ns + o];
#pragma unroll
      for (int jj = 0; jj < JMAX; ++jj) {
        int j = jg + jj * JG;
        if (j < n_t) acc[jj] += q * W[j * ns + s];
      }
    }
    bool in;
    long long node = node_of(g, cx, cy, cz, o, in);
    if (cellbuf) {
#pragma unroll
      for (int jj = 0; jj < JMAX; ++jj) {
        int j = jg + jj * JG;
        if (j < n_t) {
          const int n = g.n;
          const int lx = o % n, ly = (o / n) % n, lz = g.dim == 3 ? o / (n * n) : 0;
          cellbuf[ebuf_index(g, j, cx, cy, cz, lx, ly, lz)] = omega * acc[jj];
        }
      }
    } else if (in) {
#pragma unroll
      for (int jj = 0; jj < JMAX; ++jj) {
        int j = jg + jj * JG;
        if (j < n_t) u[(long long)j * g.nx + node] += omega * acc[jj];
      }
    }
  }
}


// ---- MFMA variant --------------------------------------------------------------------------
// 16x16x4 matrix-core products (FP64: v_mfma_f64_16x16x4f64, FP32: v_mfma_f32_16x16x4f32).
// Fragment layout on gfx950: A[i][k] in lane i + 16k, B[k][j] in lane j + 16k; the 16x16
// result D[i][j] sits in lane j + 16 (i % 4), register i / 4 for FP64 and in lane
// j + 16 (i / 4), register i % 4 for FP32.
template <class T> struct Mma;
template <> struct Mma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 fma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Mma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 fma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <class T, int NT>
__device__ inline void temporal_modes(T* P, int LD, const T* __restrict__ Tinv, long long cell, int ns,
                                      int n_t, int tid, int nthr) {
  const int c = n_t / NT;
  for (int idx = tid; idx < c * ns; idx += nthr) {
    int s = idx / c, m = idx - s * c;
    const T* Ti = Tinv + ((size_t)cell * ns + s) * NT * NT;
    T w[NT];
#pragma unroll
    for (int b = 0; b < NT; ++b) w[b] = P[s * LD + m * NT + b];
#pragma unroll
    for (int a = 0; a < NT; ++a) {
      T sacc = 0;
#pragma unroll
      for (int b = 0; b < NT; ++b) sacc += Ti[a * NT + b] * w[b];
      P[s * LD + m * NT + a] = sacc;
    }
  }
}

constexpr int MAXNT = 2;   // N tiles (NTP <= 32)
constexpr int MAXK = 32;   // K steps of 4 (NSP <= 128)

// Same map as k_asm_apply, with both products on the matrix cores.  LDS holds one
// [NSP][NTP + 1] panel: R^T (B operand of W = Q^T R^T), then W (B operand of Z = Q W),
// then Z for the write-back.  Wave w owns the 16-row tile w of both products and every N
// tile.  For the first product it loads the column strip Q(:, tile w) from global memory
// (all K steps before the first product); Q is read from global memory only there.  The
// second product needs row strips, so the column strips are handed over through two
// [16][NSP + 1] LDS chunks: in round r every wave takes the four K steps of tile r from
// chunk r, which wave r wrote one round earlier, while wave r + 1 fills the other chunk.
// The K steps are taken in the same order as from global memory, so the result does not
// depend on the hand-over.  The cell size (DIM, N) and the padded temporal width NTP are
// compile-time, so every index split is a multiply-shift; each thread keeps one local node
// and walks the temporal planes, so the node offset and its Dirichlet flag are computed once.
// one wave per 16-row tile of Q (at least four waves): BT threads
template <int NSP> constexpr int asm_threads() { return 64 * (NSP / 16 < 4 ? 4 : NSP / 16); }
// LDS bytes: the [NSP][NTP + 1] panel and two [16][NSP + 1] chunks of Q
template <class T, int NSP, int NTP> constexpr size_t asm_mfma_lds() {
  return sizeof(T) * ((size_t)NSP * (NTP + 1) + 2 * 16 * (NSP + 1));
}

template <class T, int DIM, int N, int NTP>
__global__ __launch_bounds__(512) void k_asm_mfma(
    GeomDesc g, ColourSet cs, int n_t, int nt_cell, const T* __restrict__ Q, const T* __restrict__ Tinv,
    const T* __restrict__ r, T* __restrict__ u, T omega, int nblocks, T* __restrict__ cellbuf) {
  typedef typename Mma<T>::v4 v4;
  constexpr int NS = DIM == 3 ? N * N * N : N * N;
  constexpr int NSP = (NS + 15) / 16 * 16;
  constexpr int LD = NTP + 1;
  constexpr int MT = NSP / 16, NTt = NTP / 16, KS = NSP / 4;
  constexpr int BT = asm_threads<NSP>();
  constexpr int JSTEP = BT / NSP;
  static_assert(MT <= 8 && NTt <= MAXNT && KS <= MAXK && BT % NSP == 0, "cell too large");
  constexpr int LDX = NSP + 1, XCH = 16 * LDX;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* P = reinterpret_cast<T*>(smem_raw);    // [NSP][LD]
  T* X = P + NSP * LD;                      // two [16][LDX] chunks of Q
  const long long li = xcd_swizzle(blockIdx.x, nblocks);
  if (li >= cs.count) return;
  int cx, cy, cz;
  const long long cell = colour_cell(cs, g, li, cx, cy, cz);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // this thread's local node a and temporal start j0
  const int a = tid % NSP, j0 = tid / NSP;
  bool in = false;
  long long node = 0;
  if (a < NS) {
    constexpr int p = N - 1;
    const int lx = a % N, ly = (a / N) % N, lz = DIM == 3 ? a / (N * N) : 0;
    const int gx = cx * p + lx, gy = cy * p + ly, gz = cz * p + lz;
    in = gx != 0 && gx != g.nn[0] - 1 && gy != 0 && gy != g.nn[1] - 1 &&
         (DIM == 2 || (gz != 0 && gz != g.nn[2] - 1));
    node = ((long long)gz * g.nn[1] + gy) * g.nn[0] + gx;
  }
  // P = R^T (zero padded; Dirichlet nodes read as zero); all loads issued before the stores
  {
    constexpr int JPT = NTP / JSTEP;
    T v[JPT];
#pragma unroll
    for (int jj = 0; jj < JPT; ++jj) {
      const int j = j0 + jj * JSTEP;
      v[jj] = (in && j < n_t) ? r[(long long)j * g.nx + node] : (T)0;
    }
#pragma unroll
    for (int jj = 0; jj < JPT; ++jj) P[a * LD + j0 + jj * JSTEP] = v[jj];
  }
  __syncthreads();
  const T* Qc = Q + (size_t)cell * NS * NS;    // column-major: Q(a, s) = Qc[s * NS + a]
  const int li16 = lane & 15, lk = lane >> 4;
  const int mt = wave;                          // this wave's 16-row tile of both products
  v4 acc[MAXNT];
  // this wave's column strip: av[k] = Q(4k + lk, 16 mt + li16), zero outside the cell
  T av[KS];
  // chunk layout X[s - 16 w][a], rows padded to NSP + 1 so the strided writes spread over banks
  auto put_strip = [&](T* xc) {
#pragma unroll
    for (int k = 0; k < KS; ++k) xc[li16 * LDX + 4 * k + lk] = av[k];
  };
  // W[s][j] = sum_a Q(a, s) R^T[a][j]
#pragma unroll
  for (int nt = 0; nt < NTt; ++nt) acc[nt] = v4{0, 0, 0, 0};
  if (mt < MT) {
    const int s_idx = mt * 16 + li16;
    const T* qcol = Qc + (size_t)(s_idx < NS ? s_idx : 0) * NS;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int a_idx = 4 * k + lk;
      av[k] = (s_idx < NS && a_idx < NS) ? qcol[a_idx] : (T)0;
    }
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const T* prow = P + (4 * k + lk) * LD + li16;
#pragma unroll
      for (int nt = 0; nt < NTt; ++nt) acc[nt] = Mma<T>::fma(av[k], prow[nt * 16], acc[nt]);
    }
  }
  __syncthreads();
  if (mt < MT) {
#pragma unroll
    for (int nt = 0; nt < NTt; ++nt)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) P[(mt * 16 + Mma<T>::row(lane, rr)) * LD + nt * 16 + li16] = acc[nt][rr];
  }
  if (wave == 0) put_strip(X);
  __syncthreads();
  // per mode s and time cell m: W[s, m, :] <- (lambda_s M_tau + N~)^{-1} W[s, m, :]
  switch (nt_cell) {
    case 1: temporal_modes<T, 1>(P, LD, Tinv, cell, NS, n_t, tid, BT); break;
    case 2: temporal_modes<T, 2>(P, LD, Tinv, cell, NS, n_t, tid, BT); break;
    case 3: temporal_modes<T, 3>(P, LD, Tinv, cell, NS, n_t, tid, BT); break;
    case 4: temporal_modes<T, 4>(P, LD, Tinv, cell, NS, n_t, tid, BT); break;
    case 5: temporal_modes<T, 5>(P, LD, Tinv, cell, NS, n_t, tid, BT); break;
    default: temporal_modes<T, 6>(P, LD, Tinv, cell, NS, n_t, tid, BT); break;
  }
  __syncthreads();
  // Z[a][j] = sum_s Q(a, s) W[s][j]; round r takes s in tile r from chunk r % 2
#pragma unroll
  for (int nt = 0; nt < NTt; ++nt) acc[nt] = v4{0, 0, 0, 0};
#pragma unroll 1
  for (int rd = 0; rd < MT; ++rd) {
    if (rd + 1 < MT && wave == rd + 1) put_strip(X + ((rd + 1) & 1) * XCH);
    if (mt < MT) {
      const T* xc = X + (rd & 1) * XCH;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const T aq = xc[(4 * kk + lk) * LDX + mt * 16 + li16];
        const T* prow = P + (16 * rd + 4 * kk + lk) * LD + li16;
#pragma unroll
        for (int nt = 0; nt < NTt; ++nt) acc[nt] = Mma<T>::fma(aq, prow[nt * 16], acc[nt]);
      }
    }
    __syncthreads();
  }
  // Z into LDS, then added to the interior nodes (or written to this cell's buffer slot)
  if (mt < MT) {
#pragma unroll
    for (int nt = 0; nt < NTt; ++nt)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) P[(mt * 16 + Mma<T>::row(lane, rr)) * LD + nt * 16 + li16] = acc[nt][rr];
  }
  __syncthreads();
  if (cellbuf) {
    if (a < NS) {
      const int lx = a % N, ly = (a / N) % N, lz = DIM == 3 ? a / (N * N) : 0;
      const long long e0 = ebuf_index(g, 0, cx, cy, cz, lx, ly, lz);
      const long long es = ebuf_index(g, 1, 0, 0, 0, 0, 0, 0);
#pragma unroll 4
      for (int j = j0; j < n_t; j += JSTEP) cellbuf[e0 + j * es] = omega * P[a * LD + j];
    }
  } else if (in) {
    constexpr int JPT = NTP / JSTEP;
    T v[JPT];
#pragma unroll
    for (int jj = 0; jj < JPT; ++jj) {
      const int j = j0 + jj * JSTEP;
      v[jj] = j < n_t ? u[(long long)j * g.nx + node] : (T)0;
    }
#pragma unroll
    for (int jj = 0; jj < JPT; ++jj) {
      const int j = j0 + jj * JSTEP;
      if (j < n_t) u[(long long)j * g.nx + node] = v[jj] + omega * P[a * LD + j];
    }
  }
}

template <class T, int DIM, int N, int NTP>
void launch_asm_mfma(const GeomDesc& g, const ColourSet& cs, int n_t, int nt_cell, const T* Q, const T* Tinv,
                     const T* r, T* u, T omega, hipStream_t s, T* cb) {
  constexpr int NS = DIM == 3 ? N * N * N : N * N;
  constexpr int NSP = (NS + 15) / 16 * 16;
  int nb = (int)cs.count;
  constexpr size_t lds = asm_mfma_lds<T, NSP, NTP>();
  hipLaunchKernelGGL((k_asm_mfma<T, DIM, N, NTP>), dim3(nb), dim3(asm_threads<NSP>()), lds, s,
                     g, cs, n_t, nt_cell, Q, Tinv, r, u, omega, nb, cb);
}

template <class T, int DIM, int N>
void launch_asm_mfma_nt(const GeomDesc& g, const ColourSet& cs, int n_t, int nt_cell, const T* Q, const T* Tinv,
                        const T* r, T* u, T omega, hipStream_t s, T* cb) {
  if (n_t <= 16) launch_asm_mfma<T, DIM, N, 16>(g, cs, n_t, nt_cell, Q, Tinv, r, u, omega, s, cb);
  else launch_asm_mfma<T, DIM, N, 32>(g, cs, n_t, nt_cell, Q, Tinv, r, u, omega, s, cb);
}

template <class T>
void dispatch_asm_mfma(const GeomDesc& g, const ColourSet& cs, int n_t, int nt_cell, const T* Q, const T* Tinv,
                       const T* r, T* u, T omega, hipStream_t s, T* cb) {
  if (g.dim == 3) {
    switch (g.n) {
      case 2: launch_asm_mfma_nt<T, 3, 2>(g, cs, n_t, nt_cell, Q, Tinv, r, u, omega, s, cb); break;
      case 3: launch_asm_mfma_nt<T, 3, 3>(g, cs, n_t, nt_cell, Q, Tinv, r, u, omega, s, cb); break;
      case 4: launch_asm_mfma_nt<T, 3, 4>(g, cs, n_t, nt_cell, Q, Tinv, r, u, omega, s, cb); break;
      default: launch_asm_mfma_nt<T, 3, 5>(g, cs, n_t, nt_cell, Q, Tinv, r, u, omega, s, cb); break;
    }
  } else {
    switch (g.n) {
      case 2: launch_asm_mfma_nt<T, 2, 2>(g, cs, n_t, nt_cell, Q, Tinv, r, u, omega, s, cb); break;
      case 3: launch_asm_mfma_nt<T, 2, 3>(g, cs, n_t, nt_cell, Q, Tinv, r, u, omega, s, cb); break;
      case 4: launch_asm_mfma_nt<T, 2, 4>(g, cs, n_t, nt_cell, Q, Tinv, r, u, omega, s, cb); break;
      default: launch_asm_mfma_nt<T, 2, 5>(g, cs, n_t, nt_cell, Q, Tinv, r, u, omega, s, cb); break;
    }
  }
}

}  // namespace

void asm_probe_set(const GeomDesc& g, int colour, int b, double val, double* x, hipStream_t s) {
  unsigned grid = ceil_div(g.ncells, 256);
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_probe_set, dim3(grid), dim3(256), 0, s, g, colour, b, val, x);
  STMG_CHECK_LAUNCH();
}

void asm_extract(const GeomDesc& g, int colour, int b, const double* y, double* Ablk, double* Mblk,
                 hipStream_t s) {
  int ns = (g.dim == 3) ? g.n * g.n * g.n : g.n * g.n;
  unsigned grid = ceil_div(g.ncells * ns, 256);
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_extract, dim3(grid), dim3(256), 0, s, g, colour, b, y, Ablk, Mblk);
  STMG_CHECK_LAUNCH();
}

template <class T>
void asm_tinv(long long ncells, int ns, int nt, const double* lam, const double* Mtau, const double* Nt,
              T* Tinv, int* bad, hipStream_t s) {
  unsigned grid = ceil_div(ncells * ns, 256);
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_tinv<T>, dim3(grid), dim3(256), 0, s, ncells, ns, nt, lam, Mtau, Nt, Tinv, bad);
  STMG_CHECK_LAUNCH();
}

template <class Tout>
void convert_from_double(const double* a, Tout* b, long long n, hipStream_t s) {
  unsigned grid = ceil_div(n, 256);
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL((k_convert<double, Tout>), dim3(grid), dim3(256), 0, s, a, b, n);
  STMG_CHECK_LAUNCH();
}

template <class T>
void asm_apply(const GeomDesc& g, int n_t, int nt_cell, const T* Q, const T* Tinv, const T* r, T* u,
               T omega, hipStream_t s, T* cellbuf, bool u_zero) {
  if (u_zero && !cellbuf) fail(STMG_E_ARG, "u_zero needs the per-cell buffer");
  int ns = (g.dim == 3) ? g.n * g.n * g.n : g.n * g.n;
  int JG = ABS / ns > 0 ? ABS / ns : 1;
  if ((n_t + JG - 1) / JG > JMAX) fail(STMG_E_UNSUPPORTED, "too many temporal DoFs for the smoother kernel");
  if (nt_cell > 8) fail(STMG_E_UNSUPPORTED, "too many temporal DoFs per time cell");
  size_t lds = sizeof(T) * 2 * (size_t)n_t * ns;
  const int NSP = (ns + 15) / 16 * 16, NTP = (n_t + 15) / 16 * 16;
  const bool use_mfma = n_t >= 8 && NSP <= 16 * 8 && NTP <= 16 * MAXNT && NSP <= 4 * MAXK &&
                        nt_cell <= 6;
  // colours of cells without shared nodes: block corrections are added without atomics
  // (with a per-cell buffer: every cell in one launch, then a node gather)
  const int nsets = cellbuf ? 1 : n_colours(g.dim);
  for (int colour = 0; colour < nsets; ++colour) {
    ColourSet cs = cellbuf ? all_cells(g) : colour_set(g, colour);
    if (cs.count == 0) continue;
    int nb = (int)cs.count;
    if (use_mfma)
      dispatch_asm_mfma<T>(g, cs, n_t, nt_cell, Q, Tinv, r, u, omega, s, cellbuf);
    else
      hipLaunchKernelGGL(k_asm_apply<T>, dim3(nb), dim3(ABS), lds, s, g, cs, n_t, nt_cell, Q, Tinv, r, u,
                         omega, nb, cellbuf);
    STMG_CHECK_LAUNCH();
  }
  if (cellbuf) cell_gather<T>(g, n_t, cellbuf, u, s, nullptr, u_zero);
}

template void asm_tinv<double>(long long, int, int, const double*, const double*, const double*, double*, int*, hipStream_t);
template void asm_tinv<float>(long long, int, int, const double*, const double*, const double*, float*, int*, hipStream_t);
template void convert_from_double<float>(const double*, float*, long long, hipStream_t);
template void convert_from_double<double>(const double*, double*, long long, hipStream_t);
template void asm_apply<double>(const GeomDesc&, int, int, const double*, const double*, const double*,
                                double*, double, hipStream_t, double*, bool);
template void asm_apply<float>(const GeomDesc&, int, int, const float*, const float*, const float*, float*,
                               float, hipStream_t, float*, bool);

}  // namespace stmg
