// Learned preconditioning stage (not part of the paper's method): a small 3D
// convolutional network over a slab residual, used inside FGMRES as
//     z = C(r) + V(r - S C(r)),   falling back to z = V(r) when ||r - S C(r)|| >= ||r||
// or the network output is not finite (the V-cycle judges the network).
//
// Network: s = rms(r); h_0 = r / s with one channel per temporal DoF; 3x3x3 convolutions
// with zero padding on the node lattice, ReLU between layers; C(r) = s h_L, zero on
// Dirichlet nodes.  Weights: FP32 master copy (flat, per layer W[27][C_out][C_in] then
// b[C_out]) trained with Adam; BF16 working copies W[27][CPo][CPi] and
// W^T[27][CPi][CPo] (channels padded to 16).  Activations are BF16, channels-last
// [voxel][CP]; every contraction runs on BF16 matrix cores with FP32 accumulation
// (v_mfma_f32_16x16x16_bf16: A[i][k] in lane i + 16 (k / 4), element k % 4; B[k][j] in
// lane j + 16 (k / 4); D[i][j] in lane j + 16 (i / 4), register i % 4).
#include <cmath>
#include <vector>

#include "handle.hpp"

namespace stmg {

typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16_t;

__device__ __host__ inline bf16_t to_bf16(float f) {
  union { float f; unsigned int u; } v;
  v.f = f;
  if ((v.u & 0x7f800000u) == 0x7f800000u) return (bf16_t)((v.u >> 16) | ((v.u & 0xffffu) ? 0x40u : 0u));
  unsigned int r = v.u + 0x7fffu + ((v.u >> 16) & 1u);   // round to nearest even
  return (bf16_t)(r >> 16);
}
__device__ inline float from_bf16(bf16_t b) {
  union { unsigned int u; float f; } v;
  v.u = ((unsigned int)b) << 16;
  return v.f;
}

constexpr int CMAX = 32;     // channels per layer (padded) supported by the kernels
constexpr int LMAX = 6;

struct CnnState {
  int L = 0;
  int ch[LMAX + 1] = {0};
  int cp[LMAX + 1] = {0};
  long long V = 0;           // voxels (= lattice nodes of the finest level)
  int dims[3] = {1, 1, 1};
  long long nparam = 0;
  long long woff[LMAX] = {0}, boff[LMAX] = {0};
  DevBuf theta, m, v, grad, red, lossbuf;
  DevBuf W[LMAX], Wt[LMAX], bias[LMAX];
  DevBuf act[LMAX + 1], out, g[2];
  int adam_t = 0;
};

void cnn_free(CnnState* c) { delete c; }

namespace {

enum { MODE_RELU = 0, MODE_LAST = 1, MODE_DGRAD = 2 };

__device__ inline void voxel_xyz(long long v, int nx, int ny, int& x, int& y, int& z) {
  x = (int)(v % nx);
  long long r = v / nx;
  y = (int)(r % ny);
  z = (int)(r / ny);
}

// one 16-voxel x CPO tile per wave: out[v][co] = sum_tap sum_ci in[v + off][ci] W[tap][co][ci]
template <int MODE>
__global__ __launch_bounds__(256) void k_conv(const bf16_t* __restrict__ in, int cpi,
                                              const bf16_t* __restrict__ W, int cpo,
                                              const float* __restrict__ bias, int flip,
                                              bf16_t* __restrict__ out_bf, float* __restrict__ out_f,
                                              int c_real, const bf16_t* __restrict__ mask_src, long long V,
                                              int nx, int ny, int nz) {
  const int lane = threadIdx.x & 63;
  const long long tile = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const long long v0 = tile * 16;
  if (v0 >= V) return;
  const int li = lane & 15, kb = lane >> 4;
  const long long va = v0 + li;             // voxel of this lane's A rows
  int ax = 0, ay = 0, az = 0;
  if (va < V) voxel_xyz(va, nx, ny, ax, ay, az);
  const int NT = cpo / 16, KC = cpi / 16;
  f4 acc[CMAX / 16];
#pragma unroll
  for (int n = 0; n < CMAX / 16; ++n) acc[n] = f4{0, 0, 0, 0};
  for (int tap = 0; tap < 27; ++tap) {
    int dx = tap % 3 - 1, dy = (tap / 3) % 3 - 1, dz = tap / 9 - 1;
    if (flip) { dx = -dx; dy = -dy; dz = -dz; }
    int x = ax + dx, y = ay + dy, z = az + dz;
    bool ok = va < V && x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz;
    long long nv = ok ? ((long long)z * ny + y) * nx + x : 0;
    const int wt = tap;   // flip negates the offset: g[v - off(tap)] W[tap]
    for (int kc = 0; kc < KC; ++kc) {
      bf4 a = bf4{0, 0, 0, 0};
      if (ok) a = *reinterpret_cast<const bf4*>(in + nv * cpi + kc * 16 + 4 * kb);
#pragma unroll
      for (int n = 0; n < CMAX / 16; ++n) {
        if (n >= NT) break;
        bf4 b = *reinterpret_cast<const bf4*>(W + ((size_t)wt * cpo + n * 16 + li) * cpi + kc * 16 + 4 * kb);
        acc[n] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[n], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int n = 0; n < CMAX / 16; ++n) {
    if (n >= NT) break;
    int co = n * 16 + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      long long v = v0 + 4 * kb + r;
      if (v >= V) continue;
      float val = acc[n][r];
      if (MODE == MODE_RELU) {
        val += bias[co];
        out_bf[v * cpo + co] = to_bf16(val > 0.f ? val : 0.f);
      } else if (MODE == MODE_LAST) {
        if (co < c_real) out_f[(long long)co * V + v] = val + bias[co];
      } else {
        float msk = from_bf16(mask_src[v * cpo + co]);
        out_bf[v * cpo + co] = to_bf16(msk > 0.f ? val : 0.f);
      }
    }
  }
}

// dW[tap][co][ci] += sum_v g[v][co] in[v + off(tap)][ci] over this block's voxel chunk
__global__ __launch_bounds__(256) void k_wgrad(const bf16_t* __restrict__ in, int cpi, int ci_real,
                                               const bf16_t* __restrict__ g, int cpo, int co_real,
                                               float* __restrict__ dW, long long V, int nx, int ny, int nz,
                                               int chunk) {
  const int tap = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int MT = cpo / 16, NT = cpi / 16;
  if (wave >= MT * NT) return;
  const int mt = wave / NT, nt = wave - mt * NT;
  const int dx = tap % 3 - 1, dy = (tap / 3) % 3 - 1, dz = tap / 9 - 1;
  const int li = lane & 15, kb = lane >> 4;
  long long vb = (long long)blockIdx.x * chunk;
  long long ve = vb + chunk < V ? vb + chunk : V;
  f4 acc = f4{0, 0, 0, 0};
  for (long long v0 = vb; v0 < ve; v0 += 16) {
    bf4 a, b;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      long long v = v0 + 4 * kb + e;
      short av = 0, bv = 0;
      if (v < ve) {
        av = (short)g[v * cpo + mt * 16 + li];
        int x, y, z;
        voxel_xyz(v, nx, ny, x, y, z);
        x += dx; y += dy; z += dz;
        if (x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz)
          bv = (short)in[(((long long)z * ny + y) * nx + x) * cpi + nt * 16 + li];
      }
      a[e] = av;
      b[e] = bv;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int co = mt * 16 + 4 * kb + r, ci = nt * 16 + li;
    if (co < co_real && ci < ci_real) atomicAdd(dW + ((size_t)tap * co_real + co) * ci_real + ci, acc[r]);
  }
}

__global__ void k_bgrad(const bf16_t* __restrict__ g, int cpo, int co_real, float* __restrict__ db, long long V) {
  __shared__ float sh[256];
  int co = blockIdx.y;
  float s = 0.f;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < V; v += (long long)gridDim.x * blockDim.x)
    s += from_bf16(g[v * cpo + co]);
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0 && co < co_real) atomicAdd(db + co, sh[0]);
}

// act0[v][c] = r[c][v] / s (channels-last BF16, zero padded)
__global__ void k_pack(const double* __restrict__ r, int nt, double inv_s, bf16_t* __restrict__ act, int cp,
                       long long V) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < V * cp; i += (long long)gridDim.x * blockDim.x) {
    long long v = i / cp;
    int c = (int)(i - v * cp);
    act[i] = c < nt ? to_bf16((float)(r[(long long)c * V + v] * inv_s)) : (bf16_t)0;
  }
}

// z = s * out on interior nodes, 0 on Dirichlet nodes
__global__ void k_unpack(const float* __restrict__ out, int nt, double s, const unsigned char* __restrict__ mask,
                         double* __restrict__ z, long long V) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < V * nt; i += (long long)gridDim.x * blockDim.x) {
    long long v = i % V;
    z[i] = mask[v] ? s * (double)out[i] : 0.0;
  }
}

// gL[v][c] = bf16(s * w(c, v)) with w = 2 (s out - e) / ||e||^2 (train) or w = dz (gradient probe);
// loss partial sums of (s out - e)^2 on interior nodes
__global__ void k_out_grad(const float* __restrict__ out, const double* __restrict__ e, const double* __restrict__ dz,
                           int nt, double s, double inv_ee, const unsigned char* __restrict__ mask,
                           bf16_t* __restrict__ g, int cp, long long V, double* loss) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < V * cp; i += (long long)gridDim.x * blockDim.x) {
    long long v = i / cp;
    int c = (int)(i - v * cp);
    float w = 0.f;
    if (c < nt && mask[v]) {
      long long pi = (long long)c * V + v;
      if (e) {
        double d = s * (double)out[pi] - e[pi];
        acc += d * d;
        w = (float)(s * 2.0 * d * inv_ee);
      } else {
        w = (float)(s * dz[pi]);
      }
    }
    g[i] = to_bf16(w);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) atomic_add(loss, sh[0] * inv_ee);
}

__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// BF16 working copies of one layer from the FP32 master parameters
__global__ void k_refresh(const float* __restrict__ th, long long woff, long long boff, int ci, int co, int cpi,
                          int cpo, bf16_t* __restrict__ W, bf16_t* __restrict__ Wt, float* __restrict__ b) {
  long long total = 27LL * cpo * cpi;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
    int tap = (int)(i / (cpo * cpi));
    int rem = (int)(i - (long long)tap * cpo * cpi);
    int o = rem / cpi, c = rem - o * cpi;
    float w = (o < co && c < ci) ? th[woff + ((long long)tap * co + o) * ci + c] : 0.f;
    bf16_t bw = to_bf16(w);
    W[i] = bw;
    Wt[((long long)tap * cpi + c) * cpo + o] = bw;
  }
  if (blockIdx.x == 0)
    for (int o = threadIdx.x; o < cpo; o += blockDim.x) b[o] = o < co ? th[boff + o] : 0.f;
}

inline unsigned grid_for(long long n, int bs = 256) {
  long long g = (n + bs - 1) / bs;
  if (g > 65536) g = 65536;
  return (unsigned)(g < 1 ? 1 : g);
}

void refresh(CnnState& c, hipStream_t s) {
  for (int l = 0; l < c.L; ++l) {
    hipLaunchKernelGGL(k_refresh, dim3(grid_for(27LL * c.cp[l + 1] * c.cp[l])), dim3(256), 0, s,
                       c.theta.as<float>(), c.woff[l], c.boff[l], c.ch[l], c.ch[l + 1], c.cp[l], c.cp[l + 1],
                       c.W[l].as<bf16_t>(), c.Wt[l].as<bf16_t>(), c.bias[l].as<float>());
    STMG_CHECK_LAUNCH();
  }
}

double rms_of(stmg_handle* h, const double* r, long long n) {
  norm2_check<double>(r, n, h->cnn->lossbuf.as<double>(), h->cnn->red.as<double>(), h->stream);
  std::vector<double> v = download<double>(h->cnn->lossbuf.get(), 2, h->stream);
  if (v[1] != 0.0) fail(STMG_E_NONFINITE, "non-finite values in the network input");
  return std::sqrt(v[0] / (double)n);
}

// forward through all layers; leaves activations in c.act and the FP32 output in c.out
void forward_layers(CnnState& c, hipStream_t s) {
  unsigned tiles = (unsigned)((c.V + 15) / 16);
  unsigned blocks = (tiles + 3) / 4;
  for (int l = 0; l < c.L; ++l) {
    bool last = (l == c.L - 1);
    if (!last)
      hipLaunchKernelGGL(k_conv<MODE_RELU>, dim3(blocks), dim3(256), 0, s, c.act[l].as<bf16_t>(), c.cp[l],
                         c.W[l].as<bf16_t>(), c.cp[l + 1], c.bias[l].as<float>(), 0, c.act[l + 1].as<bf16_t>(),
                         (float*)nullptr, c.ch[l + 1], (const bf16_t*)nullptr, c.V, c.dims[0], c.dims[1], c.dims[2]);
    else
      hipLaunchKernelGGL(k_conv<MODE_LAST>, dim3(blocks), dim3(256), 0, s, c.act[l].as<bf16_t>(), c.cp[l],
                         c.W[l].as<bf16_t>(), c.cp[l + 1], c.bias[l].as<float>(), 0, (bf16_t*)nullptr,
                         c.out.as<float>(), c.ch[l + 1], (const bf16_t*)nullptr, c.V, c.dims[0], c.dims[1], c.dims[2]);
    STMG_CHECK_LAUNCH();
  }
}

// back-propagate the output gradient in c.g[0] (BF16 [V][cp_L]); accumulates into c.grad
void backward_layers(CnnState& c, hipStream_t s) {
  STMG_HIP(hipMemsetAsync(c.grad.get(), 0, sizeof(float) * c.nparam, s));
  unsigned tiles = (unsigned)((c.V + 15) / 16);
  unsigned blocks = (tiles + 3) / 4;
  const int chunk = 4096;
  int cur = 0;
  for (int l = c.L - 1; l >= 0; --l) {
    bf16_t* gl = c.g[cur].as<bf16_t>();
    dim3 wg((unsigned)((c.V + chunk - 1) / chunk), 27);
    hipLaunchKernelGGL(k_wgrad, wg, dim3(256), 0, s, c.act[l].as<bf16_t>(), c.cp[l], c.ch[l], gl, c.cp[l + 1],
                       c.ch[l + 1], c.grad.as<float>() + c.woff[l], c.V, c.dims[0], c.dims[1], c.dims[2], chunk);
    STMG_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_bgrad, dim3(grid_for(c.V), c.cp[l + 1]), dim3(256), 0, s, gl, c.cp[l + 1], c.ch[l + 1],
                       c.grad.as<float>() + c.boff[l], c.V);
    STMG_CHECK_LAUNCH();
    if (l > 0) {
      // g_{l-1} = (W_l^T g_l) masked by the ReLU of layer l-1 (its output act[l] > 0)
      hipLaunchKernelGGL(k_conv<MODE_DGRAD>, dim3(blocks), dim3(256), 0, s, gl, c.cp[l + 1], c.Wt[l].as<bf16_t>(),
                         c.cp[l], (const float*)nullptr, 1, c.g[1 - cur].as<bf16_t>(), (float*)nullptr, c.ch[l],
                         c.act[l].as<bf16_t>(), c.V, c.dims[0], c.dims[1], c.dims[2]);
      STMG_CHECK_LAUNCH();
      cur = 1 - cur;
    }
  }
}

CnnState& state(stmg_handle* h) {
  if (!h->cnn) fail(STMG_E_STATE, "no network: call stmg_cnn_create first");
  return *h->cnn;
}

}  // namespace

void cnn_create(stmg_handle* h, int n_layers, const int* channels) {
  if (n_layers < 1 || n_layers > LMAX) fail(STMG_E_ARG, "n_layers must be in 1..6");
  int n_t = h->tm.n_t;
  if (channels[0] != n_t || channels[n_layers] != n_t)
    fail(STMG_E_ARG, "first and last channel counts must equal the temporal DoFs of the slab");
  if (h->levels[0]->g.dim != 3) fail(STMG_E_UNSUPPORTED, "the learned stage is implemented for 3D lattices");
  auto c = std::make_unique<CnnState>();
  c->L = n_layers;
  long long off = 0;
  for (int l = 0; l <= n_layers; ++l) {
    if (channels[l] < 1 || channels[l] > CMAX) fail(STMG_E_UNSUPPORTED, "channel counts must be in 1..32");
    c->ch[l] = channels[l];
    c->cp[l] = (channels[l] + 15) / 16 * 16;
  }
  for (int l = 0; l < n_layers; ++l) {
    c->woff[l] = off;
    off += 27LL * c->ch[l + 1] * c->ch[l];
    c->boff[l] = off;
    off += c->ch[l + 1];
  }
  c->nparam = off;
  const GeomDesc& g = h->levels[0]->g;
  c->V = g.nx;
  for (int d = 0; d < 3; ++d) c->dims[d] = g.nn[d];
  c->theta.alloc(sizeof(float) * off);
  c->m.alloc(sizeof(float) * off);
  c->v.alloc(sizeof(float) * off);
  c->grad.alloc(sizeof(float) * off);
  c->red.alloc(sizeof(double) * RED_BLOCKS * PS);
  c->lossbuf.alloc(sizeof(double) * 4);
  int cpmax = 16;
  for (int l = 0; l <= n_layers; ++l) cpmax = std::max(cpmax, c->cp[l]);
  for (int l = 0; l < n_layers; ++l) {
    c->W[l].alloc(sizeof(bf16_t) * 27 * c->cp[l + 1] * c->cp[l]);
    c->Wt[l].alloc(sizeof(bf16_t) * 27 * c->cp[l + 1] * c->cp[l]);
    c->bias[l].alloc(sizeof(float) * c->cp[l + 1]);
  }
  for (int l = 0; l < n_layers; ++l) c->act[l].alloc(sizeof(bf16_t) * c->V * c->cp[l]);
  c->out.alloc(sizeof(float) * c->V * n_t);
  c->g[0].alloc(sizeof(bf16_t) * c->V * cpmax);
  c->g[1].alloc(sizeof(bf16_t) * c->V * cpmax);
  STMG_HIP(hipMemsetAsync(c->theta.get(), 0, sizeof(float) * off, h->stream));
  STMG_HIP(hipMemsetAsync(c->m.get(), 0, sizeof(float) * off, h->stream));
  STMG_HIP(hipMemsetAsync(c->v.get(), 0, sizeof(float) * off, h->stream));
  cnn_free(h->cnn);
  h->cnn = c.release();
  refresh(*h->cnn, h->stream);
}

long long cnn_param_count(stmg_handle* h) { return state(h).nparam; }

void cnn_set_params(stmg_handle* h, const float* host, long long n) {
  CnnState& c = state(h);
  if (n != c.nparam) fail(STMG_E_ARG, "parameter count mismatch");
  for (long long i = 0; i < n; ++i)
    if (!std::isfinite(host[i])) fail(STMG_E_NONFINITE, "non-finite network parameter");
  STMG_HIP(hipMemcpyAsync(c.theta.get(), host, sizeof(float) * n, hipMemcpyHostToDevice, h->stream));
  STMG_HIP(hipMemsetAsync(c.m.get(), 0, sizeof(float) * n, h->stream));
  STMG_HIP(hipMemsetAsync(c.v.get(), 0, sizeof(float) * n, h->stream));
  c.adam_t = 0;
  refresh(c, h->stream);
  STMG_HIP(hipStreamSynchronize(h->stream));
}

void cnn_get_params(stmg_handle* h, float* host, long long n) {
  CnnState& c = state(h);
  if (n != c.nparam) fail(STMG_E_ARG, "parameter count mismatch");
  STMG_HIP(hipMemcpyAsync(host, c.theta.get(), sizeof(float) * n, hipMemcpyDeviceToHost, h->stream));
  STMG_HIP(hipStreamSynchronize(h->stream));
}

// z = C(r) for full-lattice FP64 vectors of the finest level; returns s = rms(r)
double cnn_forward(stmg_handle* h, const double* r, double* z) {
  CnnState& c = state(h);
  hipStream_t s = h->stream;
  const int n_t = h->tm.n_t;
  double sc = rms_of(h, r, c.V * n_t);
  if (sc == 0.0) {
    fill<double>(z, 0.0, c.V * n_t, s);
    return 0.0;
  }
  hipLaunchKernelGGL(k_pack, dim3(grid_for(c.V * c.cp[0])), dim3(256), 0, s, r, n_t, 1.0 / sc,
                     c.act[0].as<bf16_t>(), c.cp[0], c.V);
  STMG_CHECK_LAUNCH();
  forward_layers(c, s);
  hipLaunchKernelGGL(k_unpack, dim3(grid_for(c.V * n_t)), dim3(256), 0, s, c.out.as<float>(), n_t, sc,
                     h->levels[0]->mask.as<unsigned char>(), z, c.V);
  STMG_CHECK_LAUNCH();
  return sc;
}

// gradient of sum(dz * C(r)) with respect to the parameters (host FP32)
void cnn_param_grad(stmg_handle* h, const double* r, const double* dz, float* host) {
  CnnState& c = state(h);
  hipStream_t s = h->stream;
  const int n_t = h->tm.n_t;
  double sc = rms_of(h, r, c.V * n_t);
  STMG_HIP(hipMemsetAsync(c.grad.get(), 0, sizeof(float) * c.nparam, s));
  if (sc > 0.0) {
    hipLaunchKernelGGL(k_pack, dim3(grid_for(c.V * c.cp[0])), dim3(256), 0, s, r, n_t, 1.0 / sc,
                       c.act[0].as<bf16_t>(), c.cp[0], c.V);
    STMG_CHECK_LAUNCH();
    forward_layers(c, s);
    hipLaunchKernelGGL(k_out_grad, dim3(grid_for(c.V * c.cp[c.L])), dim3(256), 0, s, c.out.as<float>(),
                       (const double*)nullptr, dz, n_t, sc, 0.0, h->levels[0]->mask.as<unsigned char>(),
                       c.g[0].as<bf16_t>(), c.cp[c.L], c.V, (double*)nullptr);
    STMG_CHECK_LAUNCH();
    backward_layers(c, s);
  }
  STMG_HIP(hipMemcpyAsync(host, c.grad.get(), sizeof(float) * c.nparam, hipMemcpyDeviceToHost, s));
  STMG_HIP(hipStreamSynchronize(s));
}

// one Adam step on the loss ||C(r) - e||^2 / ||e||^2; returns the loss before the step
double cnn_train_step(stmg_handle* h, const double* r, const double* e, double lr) {
  CnnState& c = state(h);
  hipStream_t s = h->stream;
  const int n_t = h->tm.n_t;
  double sc = rms_of(h, r, c.V * n_t);
  double ee = rms_of(h, e, c.V * n_t);
  ee = ee * ee * (double)(c.V * n_t);
  if (sc == 0.0 || ee == 0.0) return 0.0;
  hipLaunchKernelGGL(k_pack, dim3(grid_for(c.V * c.cp[0])), dim3(256), 0, s, r, n_t, 1.0 / sc,
                     c.act[0].as<bf16_t>(), c.cp[0], c.V);
  STMG_CHECK_LAUNCH();
  forward_layers(c, s);
  STMG_HIP(hipMemsetAsync(c.lossbuf.get(), 0, sizeof(double), s));
  hipLaunchKernelGGL(k_out_grad, dim3(grid_for(c.V * c.cp[c.L])), dim3(256), 0, s, c.out.as<float>(), e,
                     (const double*)nullptr, n_t, sc, 1.0 / ee, h->levels[0]->mask.as<unsigned char>(),
                     c.g[0].as<bf16_t>(), c.cp[c.L], c.V, c.lossbuf.as<double>());
  STMG_CHECK_LAUNCH();
  backward_layers(c, s);
  c.adam_t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  float c1 = 1.f - std::pow(b1, (float)c.adam_t), c2 = 1.f - std::pow(b2, (float)c.adam_t);
  hipLaunchKernelGGL(k_adam, dim3(grid_for(c.nparam)), dim3(256), 0, s, c.theta.as<float>(), c.grad.as<float>(),
                     c.m.as<float>(), c.v.as<float>(), c.nparam, (float)lr, b1, b2, 1e-8f, c1, c2);
  STMG_CHECK_LAUNCH();
  refresh(c, s);
  return download<double>(c.lossbuf.get(), 1, s)[0];
}

// learned stage inside FGMRES (v: Arnoldi vector, z: preconditioned vector, tmp: FP64 scratch)
stmg_status cnn_precondition(stmg_handle* h, const double* v, double* z, double* tmp, bool* used) {
  hipStream_t s = h->stream;
  Level& L = *h->levels[0];
  const long long n = L.nst(h->tm.n_t);
  float* v32 = h->tmp32a.as<float>();
  float* z32 = h->tmp32b.as<float>();
  *used = false;
  double sv = cnn_forward(h, v, z);
  if (sv > 0.0) {
    vmult<double>(h, 0, z, tmp);
    axpby<double>(1.0, v, -1.0, tmp, n, s);            // tmp = v - S C(v)
    norm2_check<double>(tmp, n, h->dots.as<double>(), h->red.as<double>(), s);
    std::vector<double> rr = download<double>(h->dots.get(), 2, s);
    double vv = sv * sv * (double)n;
    if (rr[1] == 0.0 && rr[0] < vv) *used = true;
  }
  if (*used) {
    cast_d2f(tmp, v32, n, s);
    vcycle<float>(h, 0, v32, z32);
    cast_f2d(z32, tmp, n, s);
    axpy<double>(1.0, tmp, z, n, s);                   // z = C(v) + V(v - S C(v))
  } else {
    cast_d2f(v, v32, n, s);
    vcycle<float>(h, 0, v32, z32);
    cast_f2d(z32, z, n, s);
  }
  return STMG_OK;
}

}  // namespace stmg
