// Exact solve on the coarsest level (Alg. stmg, "Solve S_l u_l = f_l"): the
// interior part of the coarsest operator is probed at set-up and inverted
// densely on the host; here one thread per row applies the inverse.
#include "kernels.hpp"

namespace stmg {

namespace {
template <class T>
__global__ void k_coarse(const T* __restrict__ Cinv, const long long* __restrict__ idx, int m,
                         const T* __restrict__ f, T* __restrict__ z) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* fl = reinterpret_cast<T*>(smem_raw);
  for (int j = threadIdx.x; j < m; j += blockDim.x) fl[j] = f[idx[j]];
  __syncthreads();
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    const T* row = Cinv + (size_t)i * m;
    T s = 0;
    for (int j = 0; j < m; ++j) s += row[j] * fl[j];
    z[idx[i]] = s;
  }
}
}  // namespace

template <class T>
void coarse_apply(const T* Cinv, const long long* idx, int m, const T* f, T* z, hipStream_t s) {
  if (m <= 0) return;
  unsigned grid = ceil_div(m, 256);
  hipLaunchKernelGGL(k_coarse<T>, dim3(grid), dim3(256), sizeof(T) * m, s, Cinv, idx, m, f, z);
  STMG_CHECK_LAUNCH();
}
template void coarse_apply<double>(const double*, const long long*, int, const double*, double*, hipStream_t);
template void coarse_apply<float>(const float*, const long long*, int, const float*, float*, hipStream_t);

}  // namespace stmg
