// Vector kernels of the Krylov solver and the V-cycle (BLAS-1 style, HBM bound):
// fills, copies, axpy, casts, Dirichlet-node updates, and fused multi-vector dot
// products / updates for the Gram-Schmidt passes of FGMRES.  Reductions are two
// stage (fixed grid of partial sums, then one block per result) so results do not
// depend on atomics ordering.
#include <type_traits>

#include "kernels.hpp"

namespace stmg {

namespace {

constexpr int BS = 256;

inline unsigned grid_for(long long n) {
  long long g = (n + BS - 1) / BS;
  if (g > 65536) g = 65536;
  return (unsigned)(g < 1 ? 1 : g);
}

template <class T> __global__ void k_fill(T* y, T v, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) y[i] = v;
}
template <class T> __global__ void k_copy(const T* __restrict__ x, T* __restrict__ y, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) y[i] = x[i];
}
template <class T> __global__ void k_axpy(T a, const T* __restrict__ x, T* __restrict__ y, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) y[i] += a * x[i];
}
template <class T> __global__ void k_axpby(T a, const T* __restrict__ x, T b, T* __restrict__ y, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) y[i] = a * x[i] + b * y[i];
}
template <class T> __global__ void k_scal(T a, T* y, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) y[i] *= a;
}
__global__ void k_d2f(const double* __restrict__ x, float* __restrict__ y, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) y[i] = (float)x[i];
}
__global__ void k_f2d(const float* __restrict__ x, double* __restrict__ y, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) y[i] = (double)x[i];
}
template <class T>
__global__ void k_boundary(const int* __restrict__ bidx, long long nb, long long nx, int n_t, T a,
                           const T* __restrict__ x, T c, T* __restrict__ y) {
  long long tot = nb * n_t;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < tot; i += (long long)gridDim.x * blockDim.x) {
    long long t = i / nb, j = i - t * nb;
    long long g = t * nx + bidx[j];
    y[g] = a * x[g] + c * y[g];
  }
}

__device__ inline double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
  __syncthreads();
  return r;
}

// partial dots of up to JC vectors against w: part[block * JC + j]
// The multi-vector kernels take the vector count as a template argument, so all loads of
// one element index are issued back to back (no per-vector branches).
template <int KC>
__global__ void k_dot_part(const double* __restrict__ V, long long ldv, const double* __restrict__ w, long long n,
                           double* __restrict__ part, int self) {
  __shared__ double sh[BS / 64];
  double acc[KC];
  double ww = 0.0;
#pragma unroll
  for (int j = 0; j < KC; ++j) acc[j] = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    double wi = w[i];
    double v[KC];
#pragma unroll
    for (int j = 0; j < KC; ++j) v[j] = V[j * ldv + i];
    ww += wi * wi;
#pragma unroll
    for (int j = 0; j < KC; ++j) acc[j] += v[j] * wi;
  }
#pragma unroll
  for (int j = 0; j < KC; ++j) {
    double s = block_sum(acc[j], sh);
    if (threadIdx.x == 0) part[blockIdx.x * PS + j] = s;
  }
  if (self) {
    double s = block_sum(ww, sh);
    if (threadIdx.x == 0) part[blockIdx.x * PS + KC] = s;
  }
}

__global__ void k_dot_final(const double* __restrict__ part, int nblocks, int kc, double* out) {
  __shared__ double sh[BS / 64];
  int j = blockIdx.x;
  double v = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) v += part[b * PS + j];
  double s = block_sum(v, sh);
  if (threadIdx.x == 0) out[j] = s;
}

// w -= sum_j h[j] hs[j] V_j (hs null: 1); with NORM also the partial sums of the new ||w||^2 and a
// non-finite flag
template <int KC, bool NORM>
__global__ void k_multi_axpy_neg(const double* __restrict__ V, long long ldv, const double* __restrict__ h,
                                 const double* __restrict__ hs, double* __restrict__ w, long long n,
                                 double* __restrict__ part) {
  __shared__ double sh[BS / 64];
  double c[KC];
#pragma unroll
  for (int j = 0; j < KC; ++j) c[j] = hs ? h[j] * hs[j] : h[j];
  double acc = 0.0, bad = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    double v[KC];
#pragma unroll
    for (int j = 0; j < KC; ++j) v[j] = V[j * ldv + i];
    double s = w[i];
#pragma unroll
    for (int j = 0; j < KC; ++j) s -= c[j] * v[j];
    w[i] = s;
    if (NORM) {
      if (!isfinite(s)) bad = 1.0;
      else acc += s * s;
    }
  }
  if (NORM) {
    double a = block_sum(acc, sh);
    double b = block_sum(bad, sh);
    if (threadIdx.x == 0) { part[blockIdx.x * PS] = a; part[blockIdx.x * PS + 1] = b; }
  }
}

// K from 1 to JC, chosen at run time
template <int K, class F> void by_count(int k, F&& f) {
  if (k == K) f(std::integral_constant<int, K>{});
  else if constexpr (K > 1) by_count<K - 1>(k, f);
}

template <class T, int KC>
__global__ void k_multi_axpy_acc(const T* __restrict__ Z, long long ldz, const double* __restrict__ y,
                                 double* __restrict__ x, long long n) {
  double c[KC];
#pragma unroll
  for (int j = 0; j < KC; ++j) c[j] = y[j];
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    double v[KC];
#pragma unroll
    for (int j = 0; j < KC; ++j) v[j] = (double)Z[j * ldz + i];
    double s = x[i];
#pragma unroll
    for (int j = 0; j < KC; ++j) s += c[j] * v[j];
    x[i] = s;
  }
}

template <class T>
__global__ void k_norm_part(const T* __restrict__ x, long long n, double* part) {
  __shared__ double sh[BS / 64];
  double acc = 0.0, bad = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    double v = (double)x[i];
    if (!isfinite(v)) bad = 1.0;
    else acc += v * v;
  }
  double s = block_sum(acc, sh);
  double b = block_sum(bad, sh);
  if (threadIdx.x == 0) { part[blockIdx.x * PS] = s; part[blockIdx.x * PS + 1] = b; }
}

// grid: x = chunks of the (gx, gy) plane, y = gz, z = temporal plane.  A thread forms the up to
// 2^DIM buffer offsets of its node and their predicates, issues every load (the copies and the
// base value) and then adds the copies in a fixed cell order (predicated loads, no divergent
// loops).  The cell size is compile-time, so the cell/local splits are multiply-shifts.
template <class T, int N, int DIM>
__global__ __launch_bounds__(256) void k_cell_gather(GeomDesc g, const T* __restrict__ cb, T* y, const T* base,
                                                     int overwrite) {
  constexpr int p = N - 1;
  constexpr int NC = DIM == 3 ? 8 : 4;      // copies a node can have
  const int nn0 = g.nn[0], nn1 = g.nn[1];
  const int local = blockIdx.x * blockDim.x + threadIdx.x;
  if (local >= nn0 * nn1) return;
  const int gy = local / nn0, gx = local - gy * nn0, gz = blockIdx.y, j = blockIdx.z;
  const long long idx = ((long long)j * g.nn[2] + gz) * ((long long)nn1 * nn0) + local;
  if (gx == 0 || gx == nn0 - 1 || gy == 0 || gy == nn1 - 1 || (DIM == 3 && (gz == 0 || gz == g.nn[2] - 1))) {
    if (overwrite) y[idx] = base ? base[idx] : (T)0;
    return;
  }
  // the cell whose local index range holds the node (cx, lx), and on a face also the cell below
  // it (cx - 1, local p)
  const int cx = gx / p, lx = gx - cx * p;
  const int cy = gy / p, ly = gy - cy * p;
  const int cz = DIM == 3 ? gz / p : 0, lz = DIM == 3 ? gz - cz * p : 0;
  long long off[NC];
  bool ok[NC];
  if constexpr (N >= EBUF_CELL_MAJOR_N) {
    // [plane][cell][local node]
    constexpr int NQ = DIM == 3 ? N * N * N : N * N;
    const long long nc0 = g.nc[0], nc1 = g.nc[1];
    const long long pbase = (long long)j * g.ncells;
#pragma unroll
    for (int zz = 0; zz < (DIM == 3 ? 2 : 1); ++zz) {
      const bool zok = DIM == 2 || zz == 1 || lz == 0;
      const int czz = DIM == 3 ? (zz == 0 ? cz - 1 : cz) : 0, lzz = DIM == 3 ? (zz == 0 ? p : lz) : 0;
#pragma unroll
      for (int yy = 0; yy < 2; ++yy) {
        const bool yok = yy == 1 || ly == 0;
        const int cyy = yy == 0 ? cy - 1 : cy, lyy = yy == 0 ? p : ly;
#pragma unroll
        for (int xx = 0; xx < 2; ++xx) {
          const int k = (zz * 2 + yy) * 2 + xx;
          const int cxx = xx == 0 ? cx - 1 : cx, lxx = xx == 0 ? p : lx;
          ok[k] = zok && yok && (xx == 1 || lx == 0);
          off[k] = (pbase + ((long long)czz * nc1 + cyy) * nc0 + cxx) * NQ + (lzz * N + lyy) * N + lxx;
        }
      }
    }
  } else {
    // broken lattice
    const long long ex = (long long)g.nc[0] * N, ey = (long long)g.nc[1] * N;
    const long long ez = DIM == 3 ? (long long)g.nc[2] * N : 1;
#pragma unroll
    for (int zz = 0; zz < (DIM == 3 ? 2 : 1); ++zz) {
      const bool zok = DIM == 2 || zz == 1 || lz == 0;
      const long long zrow = DIM == 3 ? (zz == 0 ? (long long)(cz - 1) * N + p : (long long)cz * N + lz) : 0;
#pragma unroll
      for (int yy = 0; yy < 2; ++yy) {
        const bool yok = yy == 1 || ly == 0;
        const long long row = (((long long)j * ez + zrow) * ey + (yy == 0 ? (long long)(cy - 1) * N + p : (long long)cy * N + ly)) * ex;
#pragma unroll
        for (int xx = 0; xx < 2; ++xx) {
          const int k = (zz * 2 + yy) * 2 + xx;
          ok[k] = zok && yok && (xx == 1 || lx == 0);
          off[k] = row + (xx == 0 ? (long long)(cx - 1) * N + p : (long long)cx * N + lx);
        }
      }
    }
  }
  T v[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) v[k] = ok[k] ? cb[off[k]] : (T)0;
  const T b0 = overwrite ? (base ? base[idx] : (T)0) : y[idx];
  T sum = 0;
#pragma unroll
  for (int k = 0; k < NC; ++k)
    if (ok[k]) sum += v[k];
  y[idx] = b0 + sum;
}

}  // namespace

template <class T> void cell_gather(const GeomDesc& g, int n_t, const T* cb, T* y, hipStream_t s, const T* base,
                                    bool overwrite) {
  const long long plane = (long long)g.nn[0] * g.nn[1];
  const int nz = g.dim == 3 ? g.nn[2] : 1;
  if (plane * nz * n_t <= 0) return;
  if (plane > (1LL << 30) || nz > 65535 || n_t > 65535) fail(STMG_E_UNSUPPORTED, "lattice too large for the gather kernel");
  dim3 grid((unsigned)((plane + 255) / 256), (unsigned)nz, (unsigned)n_t);
  const int ow = overwrite ? 1 : 0;
#define STMG_GATHER(NN, D) hipLaunchKernelGGL((k_cell_gather<T, NN, D>), grid, dim3(256), 0, s, g, cb, y, base, ow)
  if (g.dim == 3) {
    switch (g.n) {
      case 2: STMG_GATHER(2, 3); break;
      case 3: STMG_GATHER(3, 3); break;
      case 4: STMG_GATHER(4, 3); break;
      case 5: STMG_GATHER(5, 3); break;
      default: fail(STMG_E_UNSUPPORTED, "p must be 1..4");
    }
  } else {
    switch (g.n) {
      case 2: STMG_GATHER(2, 2); break;
      case 3: STMG_GATHER(3, 2); break;
      case 4: STMG_GATHER(4, 2); break;
      case 5: STMG_GATHER(5, 2); break;
      default: fail(STMG_E_UNSUPPORTED, "p must be 1..4");
    }
  }
#undef STMG_GATHER
  STMG_CHECK_LAUNCH();
}
template void cell_gather<double>(const GeomDesc&, int, const double*, double*, hipStream_t, const double*, bool);
template void cell_gather<float>(const GeomDesc&, int, const float*, float*, hipStream_t, const float*, bool);

template <class T> void fill(T* y, T v, long long n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(BS), 0, s, y, v, n);
  STMG_CHECK_LAUNCH();
}
template <class T> void copy(const T* x, T* y, long long n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_copy<T>, dim3(grid_for(n)), dim3(BS), 0, s, x, y, n);
  STMG_CHECK_LAUNCH();
}
template <class T> void axpy(T a, const T* x, T* y, long long n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_axpy<T>, dim3(grid_for(n)), dim3(BS), 0, s, a, x, y, n);
  STMG_CHECK_LAUNCH();
}
template <class T> void axpby(T a, const T* x, T b, T* y, long long n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_axpby<T>, dim3(grid_for(n)), dim3(BS), 0, s, a, x, b, y, n);
  STMG_CHECK_LAUNCH();
}
template <class T> void scal(T a, T* y, long long n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scal<T>, dim3(grid_for(n)), dim3(BS), 0, s, a, y, n);
  STMG_CHECK_LAUNCH();
}
void cast_d2f(const double* x, float* y, long long n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_d2f, dim3(grid_for(n)), dim3(BS), 0, s, x, y, n);
  STMG_CHECK_LAUNCH();
}
void cast_f2d(const float* x, double* y, long long n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_f2d, dim3(grid_for(n)), dim3(BS), 0, s, x, y, n);
  STMG_CHECK_LAUNCH();
}
template <class T>
void boundary_axpby(const int* bidx, long long nb, long long nx, int n_t, T a, const T* x, T c, T* y,
                    hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_boundary<T>, dim3(grid_for(nb * n_t)), dim3(BS), 0, s, bidx, nb, nx, n_t, a, x, c, y);
  STMG_CHECK_LAUNCH();
}

void multi_dot(const double* V, long long ldv, int k, const double* w, long long n, double* out,
               double* part, hipStream_t s, bool self) {
  unsigned nb = grid_for(n);
  if (nb > RED_BLOCKS) nb = RED_BLOCKS;
  for (int j0 = 0; j0 < k; j0 += JC) {
    int kc = k - j0 < JC ? k - j0 : JC;
    int sf = (self && j0 + kc == k) ? 1 : 0;     // w . w with the last group, into out[k]
    by_count<JC>(kc, [&](auto K) {
      hipLaunchKernelGGL((k_dot_part<decltype(K)::value>), dim3(nb), dim3(BS), 0, s, V + j0 * ldv, ldv, w, n, part, sf);
    });
    STMG_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_dot_final, dim3(kc + sf), dim3(BS), 0, s, part, (int)nb, kc + sf, out + j0);
    STMG_CHECK_LAUNCH();
  }
}

void multi_axpy_neg(const double* V, long long ldv, int k, const double* h, double* w, long long n,
                    hipStream_t s) {
  if (n <= 0 || k <= 0) return;
  for (int j0 = 0; j0 < k; j0 += JC) {
    int kc = k - j0 < JC ? k - j0 : JC;
    by_count<JC>(kc, [&](auto K) {
      hipLaunchKernelGGL((k_multi_axpy_neg<decltype(K)::value, false>), dim3(grid_for(n)), dim3(BS), 0, s,
                         V + j0 * ldv, ldv, h + j0, (const double*)nullptr, w, n, (double*)nullptr);
    });
    STMG_CHECK_LAUNCH();
  }
}

void multi_axpy_neg_norm(const double* V, long long ldv, int k, const double* h, double* w, long long n,
                         double* out, double* part, hipStream_t s, const double* hs) {
  unsigned nb = grid_for(n);
  if (nb > RED_BLOCKS) nb = RED_BLOCKS;
  for (int j0 = 0; j0 < k; j0 += JC) {
    int kc = k - j0 < JC ? k - j0 : JC;
    const bool last = j0 + kc == k;
    by_count<JC>(kc, [&](auto K) {
      if (last)
        hipLaunchKernelGGL((k_multi_axpy_neg<decltype(K)::value, true>), dim3(nb), dim3(BS), 0, s,
                           V + j0 * ldv, ldv, h + j0, hs ? hs + j0 : hs, w, n, part);
      else
        hipLaunchKernelGGL((k_multi_axpy_neg<decltype(K)::value, false>), dim3(grid_for(n)), dim3(BS), 0, s,
                           V + j0 * ldv, ldv, h + j0, hs ? hs + j0 : hs, w, n, (double*)nullptr);
    });
    STMG_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_dot_final, dim3(2), dim3(BS), 0, s, part, (int)nb, 2, out);
  STMG_CHECK_LAUNCH();
}

template <class T>
void multi_axpy_acc(const T* Z, long long ldz, int k, const double* y, double* x, long long n,
                    hipStream_t s) {
  if (n <= 0 || k <= 0) return;
  for (int j0 = 0; j0 < k; j0 += JC) {
    int kc = k - j0 < JC ? k - j0 : JC;
    by_count<JC>(kc, [&](auto K) {
      hipLaunchKernelGGL((k_multi_axpy_acc<T, decltype(K)::value>), dim3(grid_for(n)), dim3(BS), 0, s,
                         Z + j0 * ldz, ldz, y + j0, x, n);
    });
    STMG_CHECK_LAUNCH();
  }
}

template <class T> void norm2_check(const T* x, long long n, double* out, double* part, hipStream_t s) {
  unsigned nb = grid_for(n);
  if (nb > RED_BLOCKS) nb = RED_BLOCKS;
  hipLaunchKernelGGL(k_norm_part<T>, dim3(nb), dim3(BS), 0, s, x, n, part);
  STMG_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_dot_final, dim3(2), dim3(BS), 0, s, part, (int)nb, 2, out);
  STMG_CHECK_LAUNCH();
}

#define INST(T)                                                                                   \
  template void fill<T>(T*, T, long long, hipStream_t);                                            \
  template void copy<T>(const T*, T*, long long, hipStream_t);                                     \
  template void axpy<T>(T, const T*, T*, long long, hipStream_t);                                  \
  template void axpby<T>(T, const T*, T, T*, long long, hipStream_t);                              \
  template void scal<T>(T, T*, long long, hipStream_t);                                            \
  template void boundary_axpby<T>(const int*, long long, long long, int, T, const T*, T, T*,      \
                                  hipStream_t);                                                    \
  template void multi_axpy_acc<T>(const T*, long long, int, const double*, double*, long long,    \
                                  hipStream_t);                                                    \
  template void norm2_check<T>(const T*, long long, double*, double*, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace stmg
