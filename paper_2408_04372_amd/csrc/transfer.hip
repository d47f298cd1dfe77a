// Spatial grid transfers (Section 3.2).  On the structured lattice the
// prolongation is a Kronecker product of 1D interpolation matrices
// (P = P_z (x) P_y (x) P_x, applied to every temporal plane, "P^h (x) u"), so it is
// applied as d one-dimensional sweeps; the restriction R = P^T uses the transposed
// 1D matrices.  Dirichlet rows and columns are already removed from the 1D factors.  Each sweep is a banded 1D contraction with unit-stride access
// along x, so consecutive lanes read consecutive addresses in every direction.
//
// Temporal transfers (k- and tau-coarsening, Section 3.2) act on the temporal index only,
// "I (x) P^tau": every interior node x maps its n_c coarse temporal values to n_f fine ones
// with the dense (n_f x n_c) matrix P_t, or back with P_t^T; Dirichlet nodes carry zero.
#include "kernels.hpp"

namespace stmg {

namespace {

// grid: x = chunks of the (i0, i1) output plane, y = i2, z = temporal plane; 32-bit index math.
// STAGED: the 1D matrix (len rows, nnz entries) is copied to LDS once per block.
template <class T, bool STAGED, int KMAX>
__global__ __launch_bounds__(256) void k_sweep(const T* __restrict__ in, T* __restrict__ out, int d0, int d1, int d2,
                                               int ax, int o0, int o1, const int* __restrict__ ptr,
                                               const int* __restrict__ col, const T* __restrict__ w,
                                               int accumulate, int len, int nnz) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int* P = ptr;
  const int* C = col;
  const T* W = w;
  if constexpr (STAGED) {
    T* sw = reinterpret_cast<T*>(smem_raw);
    int* sptr = reinterpret_cast<int*>(sw + nnz);
    int* scol = sptr + len + 1;
    for (int e = threadIdx.x; e <= len; e += blockDim.x) sptr[e] = ptr[e];
    for (int e = threadIdx.x; e < nnz; e += blockDim.x) { scol[e] = col[e]; sw[e] = w[e]; }
    __syncthreads();
    P = sptr;
    C = scol;
    W = sw;
  }
  const int local = blockIdx.x * blockDim.x + threadIdx.x;
  if (local >= o0 * o1) return;
  const int i0 = local % o0, i1 = local / o0, i2 = blockIdx.y, t = blockIdx.z;
  const int o2 = gridDim.y;
  const long long plane_out = (long long)o0 * o1 * o2;
  const long long plane_in = (long long)d0 * d1 * d2;
  const long long r = (long long)i2 * o0 * o1 + local;
  const int ia = ax == 0 ? i0 : (ax == 1 ? i1 : i2);
  // the input line through this output point; the contracted index moves with stride st
  const long long st = ax == 0 ? 1 : (ax == 1 ? (long long)d0 : (long long)d0 * d1);
  const long long line = ax == 0 ? ((long long)i2 * d1 + i1) * d0
                                  : (ax == 1 ? (long long)i2 * d1 * d0 + i0 : (long long)i1 * d0 + i0);
  const T* src = in + t * plane_in + line;
  T s = 0;
  const int k0 = P[ia], k1 = P[ia + 1];
  if (KMAX > 0) {
    // at most KMAX entries per row: every load of the row is issued before the first use
    T v[KMAX > 0 ? KMAX : 1], c[KMAX > 0 ? KMAX : 1];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
      const int k = k0 + q;
      c[q] = k < k1 ? W[k] : (T)0;
      v[q] = k < k1 ? src[C[k] * st] : (T)0;
    }
#pragma unroll
    for (int q = 0; q < KMAX; ++q) s += c[q] * v[q];
  } else {
    for (int k = k0; k < k1; ++k) s += W[k] * src[C[k] * st];
  }
  T* dst = out + t * plane_out + r;
  if (accumulate) *dst += s;
  else *dst = s;
}

// one thread per lattice node: load the node's input planes (coalesced over x), write every
// output plane.  P (nf x nc, row-major) is staged in LDS.
template <class T>
__global__ __launch_bounds__(256) void k_time_transfer(const T* __restrict__ P, int nf, int nc, long long nx,
                                                       const unsigned char* __restrict__ mask,
                                                       const T* __restrict__ in, T* __restrict__ out, int mode) {
  __shared__ T Ps[TT_MAX * TT_MAX];
  for (int i = threadIdx.x; i < nf * nc; i += blockDim.x) Ps[i] = P[i];
  __syncthreads();
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= nx) return;
  const bool inner = mask[x] != 0;
  const int nin = mode == 2 ? nf : nc, nout = mode == 2 ? nc : nf;
  T v[TT_MAX];
  for (int j = 0; j < nin; ++j) v[j] = inner ? in[(long long)j * nx + x] : (T)0;
  for (int i = 0; i < nout; ++i) {
    T s = 0;
    if (mode == 2)
      for (int j = 0; j < nin; ++j) s += Ps[j * nc + i] * v[j];      // P^T
    else
      for (int j = 0; j < nin; ++j) s += Ps[i * nc + j] * v[j];      // P
    T* dst = out + (long long)i * nx + x;
    if (mode == 1) *dst += s;
    else *dst = s;
  }
}

// Fused tensor-product transfer: out (+)= (Az (x) Ay (x) Ax) in on every temporal plane.  A
// workgroup owns TX x TY output nodes of one plane in x and y (one per thread) and a chunk of TZC
// output z planes, and streams through the input z planes the chunk depends on: each input plane's
// patch (SY x SX nodes, prefetched into registers while the previous plane is contracted) is staged
// in LDS, contracted along x and y, and added into the TZC accumulators of every thread with the
// chunk's dense z weights.  Every input node is read once per tile column (plus the x-y halo) and
// every output node written once; the three sweeps of sweep1d and their intermediate vectors are
// gone.  Tile ranges, padded rows and the z weights come from host-built tables.
constexpr int T3_PF = 8;                 // patch values per thread (patch <= 8 * 256 nodes)

template <class T, int KMAX, int TZC>
__global__ __launch_bounds__(256) void k_tensor3(const T* __restrict__ in, T* __restrict__ out, int in0, int in1,
                                                 int in2, int out0, int out1, int out2, T3Axis ax, T3Axis ay, T3Axis az,
                                                 int lgx, int TY, int SX, int SZ, int ntx, int nty, int accumulate) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int TX = 1 << lgx;
  const int tid = threadIdx.x;
  const int tile = blockIdx.x, txi = tile % ntx, tyz = tile / ntx, tyi = tyz % nty, tzi = tyz / nty;
  const int ox0 = txi << lgx, oy0 = tyi * TY, oz0 = tzi * TZC;
  const int fx = tid & (TX - 1), fy = tid >> lgx;
  const bool own = fy < TY && ox0 + fx < out0 && oy0 + fy < out1;
  T* dst = out + (long long)blockIdx.y * out0 * out1 * out2 + ((long long)oz0 * out1 + (oy0 + fy)) * out0 + (ox0 + fx);
  const long long zstride = (long long)out0 * out1;
  const int lx = ax.lo[txi], ly = ay.lo[tyi], lz = az.lo[tzi];
  const int bx = ax.hi[txi] - lx + 1, by = ay.hi[tyi] - ly + 1, bz = az.hi[tzi] - lz + 1;
  T acc[TZC];
#pragma unroll
  for (int k = 0; k < TZC; ++k) acc[k] = 0;
  if (bx > 0 && by > 0 && bz > 0) {
    T* blk = reinterpret_cast<T*>(smem_raw);               // [by][SX] input patch
    T* t1 = blk + (size_t)by * SX;                          // [by][TX]
    const T* src = in + (long long)blockIdx.y * ((long long)in0 * in1 * in2) + ((long long)lz * in1 + ly) * in0 + lx;
    // patch offsets of this thread (fixed for every input plane)
    int goff[T3_PF], loff[T3_PF];
    const int np = bx * by;
#pragma unroll
    for (int k = 0; k < T3_PF; ++k) {
      const int e = tid + k * 256;
      const int r = e / bx, ix = e - r * bx;
      goff[k] = r * in0 + ix;
      loff[k] = e < np ? r * SX + ix : -1;
    }
    // rows of Ax and Ay for this thread
    T wx[KMAX], wy[KMAX];
    int cx[KMAX], cy[KMAX];
    const int rx = ox0 + fx, ry = oy0 + fy;
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
      wx[q] = rx < out0 ? static_cast<const T*>(ax.w)[(size_t)rx * KMAX + q] : (T)0;
      cx[q] = rx < out0 ? ax.col[(size_t)rx * KMAX + q] : 0;
      wy[q] = own ? static_cast<const T*>(ay.w)[(size_t)ry * KMAX + q] : (T)0;
      cy[q] = own ? ay.col[(size_t)ry * KMAX + q] : 0;
    }
    const T* zw = static_cast<const T*>(az.w) + (size_t)tzi * TZC * SZ;   // [TZC][SZ] dense z weights
    const long long pstride = (long long)in0 * in1;
    T pv[T3_PF];
#pragma unroll
    for (int k = 0; k < T3_PF; ++k) pv[k] = loff[k] >= 0 ? src[goff[k]] : (T)0;
    for (int iz = 0; iz < bz; ++iz) {
#pragma unroll
      for (int k = 0; k < T3_PF; ++k)
        if (loff[k] >= 0) blk[loff[k]] = pv[k];
      if (iz + 1 < bz) {
        const T* nsrc = src + (iz + 1) * pstride;
#pragma unroll
        for (int k = 0; k < T3_PF; ++k) pv[k] = loff[k] >= 0 ? nsrc[goff[k]] : (T)0;
      }
      __syncthreads();
      for (int e = tid; e < by * TX; e += 256) {
        const T* b = blk + (size_t)(e >> lgx) * SX;
        T a = 0;
#pragma unroll
        for (int q = 0; q < KMAX; ++q) a += wx[q] * b[cx[q]];
        t1[e] = a;
      }
      __syncthreads();
      if (own) {
        T v = 0;
#pragma unroll
        for (int q = 0; q < KMAX; ++q) v += wy[q] * t1[(size_t)cy[q] * TX + fx];
#pragma unroll
        for (int k = 0; k < TZC; ++k) acc[k] += zw[k * SZ + iz] * v;
      }
    }
  }
  if (own) {
    const int kl = out2 - 1 - oz0;                           // last plane of the chunk inside the lattice
    if (accumulate) {
      // every old value is loaded before the first store (planes past the lattice reload the last one)
      T old[TZC];
#pragma unroll
      for (int k = 0; k < TZC; ++k) old[k] = dst[(k < kl ? k : kl) * zstride];
#pragma unroll
      for (int k = 0; k < TZC; ++k) acc[k] += old[k];
    }
#pragma unroll
    for (int k = 0; k < TZC; ++k)
      if (k <= kl) dst[k * zstride] = acc[k];
  }
}

}  // namespace

template <class T>
void tensor3(const T* in, T* out, int n_t, const int in_dims[3], const int out_dims[3], const Tensor3Plan& pl,
             const T3Axis ax[3], bool accumulate, hipStream_t s) {
  if ((long long)out_dims[0] * out_dims[1] * out_dims[2] * n_t <= 0) return;
  if (!pl.ok) fail(STMG_E_STATE, "fused transfer without a plan");
  const long long tiles = (long long)pl.nt[0] * pl.nt[1] * pl.nt[2];
  if (tiles >= (1LL << 24) || n_t > 65535) fail(STMG_E_UNSUPPORTED, "lattice too large for the transfer kernel");
  if (pl.T[0] * pl.T[1] > 256 || (1 << pl.lg[0]) != pl.T[0] || pl.S[0] * pl.S[1] > T3_PF * 256)
    fail(STMG_E_STATE, "fused transfer tile");
  const size_t lds = sizeof(T) * ((size_t)pl.S[1] * pl.S[0] + (size_t)pl.S[1] * pl.T[0]);
  dim3 grid((unsigned)tiles, (unsigned)n_t);
  const int acc = accumulate ? 1 : 0;
#define STMG_T3(K, Z) hipLaunchKernelGGL((k_tensor3<T, K, Z>), grid, dim3(256), lds, s, in, out, in_dims[0], in_dims[1], \
                                         in_dims[2], out_dims[0], out_dims[1], out_dims[2], ax[0], ax[1], ax[2], \
                                         pl.lg[0], pl.T[1], pl.S[0], pl.S[2], pl.nt[0], pl.nt[1], acc)
#define STMG_T3K(Z)                      \
  switch (pl.kmax) {                     \
    case 2: STMG_T3(2, Z); break;        \
    case 3: STMG_T3(3, Z); break;        \
    case 4: STMG_T3(4, Z); break;        \
    case 5: STMG_T3(5, Z); break;        \
    case 6: STMG_T3(6, Z); break;        \
    case 8: STMG_T3(8, Z); break;        \
    case 10: STMG_T3(10, Z); break;      \
    default: fail(STMG_E_UNSUPPORTED, "transfer row length"); \
  }
  if (pl.T[2] == 16) { STMG_T3K(16) }
  else if (pl.T[2] == 4) { STMG_T3K(4) }
  else fail(STMG_E_STATE, "fused transfer z chunk");
#undef STMG_T3K
#undef STMG_T3
  STMG_CHECK_LAUNCH();
}

template void tensor3<double>(const double*, double*, int, const int*, const int*, const Tensor3Plan&,
                              const T3Axis*, bool, hipStream_t);
template void tensor3<float>(const float*, float*, int, const int*, const int*, const Tensor3Plan&,
                             const T3Axis*, bool, hipStream_t);

template <class T>
void time_transfer(const T* P, int nf, int nc, long long nx, const unsigned char* mask, const T* in, T* out,
                   int mode, hipStream_t s) {
  if (nf < 1 || nc < 1 || nf > TT_MAX || nc > TT_MAX) fail(STMG_E_UNSUPPORTED, "too many temporal DoFs for the temporal transfer");
  if (mode < 0 || mode > 2) fail(STMG_E_ARG, "temporal transfer mode");
  if (nx <= 0) return;
  hipLaunchKernelGGL(k_time_transfer<T>, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, s, P, nf, nc, nx, mask,
                     in, out, mode);
  STMG_CHECK_LAUNCH();
}

template void time_transfer<double>(const double*, int, int, long long, const unsigned char*, const double*,
                                    double*, int, hipStream_t);
template void time_transfer<float>(const float*, int, int, long long, const unsigned char*, const float*, float*,
                                   int, hipStream_t);

template <class T>
void sweep1d(const T* in, T* out, int n_t, const int in_dims[3], int ax, int out_len, const int* ptr,
             const int* col, const T* w, int nnz, int max_row, bool accumulate, hipStream_t s) {
  const int o0 = ax == 0 ? out_len : in_dims[0], o1 = ax == 1 ? out_len : in_dims[1],
            o2 = ax == 2 ? out_len : in_dims[2];
  if ((long long)o0 * o1 * o2 * n_t <= 0) return;
  if ((long long)o0 * o1 > (1LL << 30) || o2 > 65535 || n_t > 65535) fail(STMG_E_UNSUPPORTED, "lattice too large for the transfer kernel");
  dim3 grid((unsigned)((o0 * o1 + 255) / 256), (unsigned)o2, (unsigned)n_t);
  const size_t lds = sizeof(T) * (size_t)nnz + sizeof(int) * (size_t)(out_len + 1 + nnz);
  const bool staged = lds <= 16 * 1024;
  const int acc = accumulate ? 1 : 0;
#define STMG_SWEEP(ST, K) hipLaunchKernelGGL((k_sweep<T, ST, K>), grid, dim3(256), ST ? lds : 0, s, in, out, in_dims[0], \
                                            in_dims[1], in_dims[2], ax, o0, o1, ptr, col, w, acc, out_len, nnz)
  if (staged) {
    if (max_row <= 4) STMG_SWEEP(true, 4);
    else if (max_row <= 8) STMG_SWEEP(true, 8);
    else if (max_row <= 12) STMG_SWEEP(true, 12);
    else STMG_SWEEP(true, 0);
  } else {
    if (max_row <= 4) STMG_SWEEP(false, 4);
    else if (max_row <= 8) STMG_SWEEP(false, 8);
    else if (max_row <= 12) STMG_SWEEP(false, 12);
    else STMG_SWEEP(false, 0);
  }
#undef STMG_SWEEP
  STMG_CHECK_LAUNCH();
}

template void sweep1d<double>(const double*, double*, int, const int*, int, int, const int*, const int*,
                              const double*, int, int, bool, hipStream_t);
template void sweep1d<float>(const float*, float*, int, const int*, int, int, const int*, const int*,
                             const float*, int, int, bool, hipStream_t);

}  // namespace stmg
