// Spatial grid transfers (Section 3.2).  On the structured lattice the
// prolongation is a Kronecker product of 1D interpolation matrices
// (P = P_z (x) P_y (x) P_x, applied to every temporal plane, "P^h (x) u"), so it is
// applied as d one-dimensional sweeps; the restriction R = P^T uses the transposed
// 1D matrices.  Each sweep is a banded 1D contraction with unit-stride access
// along x, so consecutive lanes read consecutive addresses in every direction.
#include "kernels.hpp"

namespace stmg {

namespace {

template <class T>
__global__ void k_sweep(const T* __restrict__ in, T* __restrict__ out, int n_t, int d0, int d1, int d2,
                        int ax, int out_len, const int* __restrict__ ptr, const int* __restrict__ col,
                        const T* __restrict__ w, const unsigned char* __restrict__ mask_in,
                        const unsigned char* __restrict__ mask_out, int accumulate) {
  int o0 = ax == 0 ? out_len : d0, o1 = ax == 1 ? out_len : d1, o2 = ax == 2 ? out_len : d2;
  long long plane_out = (long long)o0 * o1 * o2;
  long long plane_in = (long long)d0 * d1 * d2;
  long long total = plane_out * n_t;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    long long t = idx / plane_out;
    long long r = idx - t * plane_out;
    int i0 = (int)(r % o0);
    int i1 = (int)((r / o0) % o1);
    int i2 = (int)(r / ((long long)o0 * o1));
    int ia = ax == 0 ? i0 : (ax == 1 ? i1 : i2);
    T s = 0;
    if (!mask_out || mask_out[r]) {
      for (int k = ptr[ia]; k < ptr[ia + 1]; ++k) {
        int c = col[k];
        int j0 = ax == 0 ? c : i0, j1 = ax == 1 ? c : i1, j2 = ax == 2 ? c : i2;
        long long sidx = ((long long)j2 * d1 + j1) * d0 + j0;
        if (mask_in && !mask_in[sidx]) continue;
        s += w[k] * in[t * plane_in + sidx];
      }
    }
    if (accumulate) out[idx] += s;
    else out[idx] = s;
  }
}

}  // namespace

template <class T>
void sweep1d(const T* in, T* out, int n_t, const int in_dims[3], int ax, int out_len, const int* ptr,
             const int* col, const T* w, const unsigned char* mask_in, const unsigned char* mask_out,
             bool accumulate, hipStream_t s) {
  long long o = (long long)(ax == 0 ? out_len : in_dims[0]) * (ax == 1 ? out_len : in_dims[1]) *
                (ax == 2 ? out_len : in_dims[2]) * n_t;
  if (o <= 0) return;
  long long g = (o + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_sweep<T>, dim3((unsigned)g), dim3(256), 0, s, in, out, n_t, in_dims[0],
                     in_dims[1], in_dims[2], ax, out_len, ptr, col, w, mask_in, mask_out,
                     accumulate ? 1 : 0);
  STMG_CHECK_LAUNCH();
}

template void sweep1d<double>(const double*, double*, int, const int*, int, int, const int*, const int*,
                              const double*, const unsigned char*, const unsigned char*, bool, hipStream_t);
template void sweep1d<float>(const float*, float*, int, const int*, int, int, const int*, const int*,
                             const float*, const unsigned char*, const unsigned char*, bool, hipStream_t);

}  // namespace stmg
