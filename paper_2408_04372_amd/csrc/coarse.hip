// Exact solve on the coarsest level (Alg. stmg, "Solve S_l u_l = f_l"): the
// interior part of the coarsest operator is probed at set-up and inverted
// densely on the host; here one wave per row applies the inverse (lanes read the
// row-major inverse contiguously, then a fixed-order wave reduction).
#include <algorithm>

#include "kernels.hpp"

namespace stmg {

namespace {
template <class T>
__global__ __launch_bounds__(1024) void k_coarse(const T* __restrict__ Cinv, const long long* __restrict__ idx, int m,
                                                 const T* __restrict__ f, T* __restrict__ z) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* fl = reinterpret_cast<T*>(smem_raw);
  for (int j = threadIdx.x; j < m; j += blockDim.x) fl[j] = f[idx[j]];
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  for (int i = blockIdx.x * nw + wave; i < m; i += gridDim.x * nw) {
    const T* row = Cinv + (size_t)i * m;
    T s = 0;
    for (int j = lane; j < m; j += 64) s += row[j] * fl[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) z[idx[i]] = s;
  }
}
}  // namespace

template <class T>
void coarse_apply(const T* Cinv, const long long* idx, int m, const T* f, T* z, hipStream_t s) {
  if (m <= 0) return;
  const int rows_per_block = 16;
  const unsigned grid = std::min(ceil_div((size_t)m, rows_per_block), 256u);
  hipLaunchKernelGGL(k_coarse<T>, dim3(grid), dim3(64 * rows_per_block), sizeof(T) * m, s, Cinv, idx, m, f, z);
  STMG_CHECK_LAUNCH();
}
template void coarse_apply<double>(const double*, const long long*, int, const double*, double*, hipStream_t);
template void coarse_apply<float>(const float*, const long long*, int, const float*, float*, hipStream_t);

}  // namespace stmg
