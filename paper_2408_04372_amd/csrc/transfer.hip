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

}  // namespace

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
