// Brick-tiled matrix-free space-time operator for Cartesian levels with one coefficient per cell:
//   y = base + scale * (M_T (x) A_h + N_T (x) M_h) x     (overwrite), or   y += scale * (...) x
// on interior rows (Section 3.1: the cell operators are formed once per temporal DoF by sum
// factorisation and the temporal factors are small dense matrices).
//
// On an axis-aligned box cell with widths (h_x, h_y, h_z) and constant coefficient rho the cell
// matrices factor into 1D reference matrices on [0, 1] (GLL nodal basis, exact Gauss quadrature):
//   M_K = h_x h_y h_z  Mz (x) My (x) Mx,
//   A_K = rho [ (h_y h_z / h_x) Mz My Kx + (h_x h_z / h_y) Mz Ky Mx + (h_x h_y / h_z) Kz My Mx ],
// so the fused evaluation  A_K a_i + M_K b_i  (a_i = (M_T x)_i, b_i = (N_T x)_i at the nodes) takes
// eight 1D sweeps per (cell, temporal DoF) instead of twelve sweeps plus quadrature-point work:
//   U = Mx a,  V = sx Kx a + sm Mx b,   W = Mz V + sz Kz U,  Z = Mz U,   Y = My W + sy Ky Z.
//
// MI355X mapping (brick tiling in brick.hpp).  A team of N = p+1 lanes (teams never straddle a
// wave) owns one (cell, output temporal DoF); lane t first holds the y = t plane of the cell
// ([z][x]: x and z sweeps are lane local), then, after a per-x-slice exchange through a small LDS
// scratch, the z = t plane ([y][x]: y sweeps lane local).
#include <type_traits>

#include "brick.hpp"

namespace stmg {

namespace {

// The 1D mass and stiffness matrices are symmetric and centrosymmetric (GLL nodes and Gauss points
// are symmetric about 1/2), so entry (i, j) equals (j, i) and (N-1-j, N-1-i).  Reading every entry
// through its canonical representative leaves (N^2 + N)/4-ish distinct values per matrix, which the
// unrolled sweeps keep in scalar registers.
template <int N>
__host__ __device__ constexpr int sym_row(int i, int j) {
  const int a = i < j ? i : j, b = i < j ? j : i;
  const int a2 = N - 1 - b, b2 = N - 1 - a;
  return (a < a2 || (a == a2 && b <= b2)) ? a : a2;
}
template <int N>
__host__ __device__ constexpr int sym_col(int i, int j) {
  const int a = i < j ? i : j, b = i < j ? j : i;
  const int a2 = N - 1 - b, b2 = N - 1 - a;
  return (a < a2 || (a == a2 && b <= b2)) ? b : b2;
}
#define SYM(Mat, i, j) (Mat)[sym_row<N>((i), (j))][sym_col<N>((i), (j))]

template <class T, int N>
struct BrickOpArgs {
  T M[N][N];          // 1D reference mass
  T K[N][N];          // 1D reference stiffness
  T sx, sy, sz, sm;   // h_y h_z / h_x, h_x h_z / h_y, h_x h_y / h_z, h_x h_y h_z
  GeomDesc g;
  TemporalDev<T> tp;
  const T* x;
  T* y;
  const T* base;      // overwrite mode: added once per node (null: zero)
  T scale;
  int overwrite;
  BrickLaunch L;
};

template <class T, int N>
__global__ __launch_bounds__(512) void st_apply3_brick(BrickOpArgs<T, N> A) {
  constexpr int p = N - 1;
  // global loads in flight per thread in the stage and write-back (measured on 128^3 Q4 and Q2
  // levels: 24 for Q4, whose compute phase sets the register count anyway, 8 for lower degrees)
  constexpr int OP_BATCH = N >= 5 ? 24 : 8;
  constexpr int TPW = 64 / N;           // teams per wave
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const GeomDesc& g = A.g;
  const int n_t = A.tp.n_t;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int nbx = A.L.NBd[0], nby = A.L.NBd[1];
  const BrickPos P = brick_pos(A.L, g);
  const int NB = P.NB;
  const int teams = (nthr >> 6) * TPW;
  const int ncx = P.nc[0], ncy = P.nc[1], ncz = P.nc[2];
  const int c0x = P.c0[0], c0y = P.c0[1], c0z = P.c0[2];

  // [n_t][NB]: input, then the exchange slices of phase 2 ([teams][2][N][N]), then the brick's sums
  T* xs = reinterpret_cast<T*>(smem_raw);
  T* scr = xs;
  T* zl = xs + (size_t)max(n_t * NB, teams * 2 * N * N);   // one zero
  // rows of M_T and N_T on their union pattern: x_j is read once for both products
  const int unnz = A.tp.unnz;
  T* um_s = zl + 1;
  T* un_s = um_s + unnz;
  int* uptr_s = reinterpret_cast<int*>(un_s + unnz);
  int* ucol_s = uptr_s + n_t + 1;
  for (int e = tid; e < unnz; e += nthr) { um_s[e] = A.tp.umval[e]; un_s[e] = A.tp.unval[e]; ucol_s[e] = A.tp.ucol[e]; }
  for (int e = tid; e <= n_t; e += nthr) uptr_s[e] = A.tp.uptr[e];
  if (tid == 0) *zl = (T)0;

  brick_stage<T, OP_BATCH>(g, A.L, P, n_t, A.x, xs);
  __syncthreads();

  const int wave = tid >> 6, lane = tid & 63;
  const int tw = lane / N, t = lane - tw * N;
  const int team = wave * TPW + tw;
  const int ncell = ncx * ncy * ncz;
  const bool act = tw < TPW && team < ncell * n_t;
  const int lc = act ? team / n_t : 0, i = act ? team - lc * n_t : 0;
  const int lcx = lc % ncx, lcy = (lc / ncx) % ncy, lcz = lc / (ncx * ncy);
  const long long cell = ((long long)(c0z + lcz) * g.nc[1] + (c0y + lcy)) * g.nc[0] + (c0x + lcx);
  const T rho = (act && g.rho) ? (T)g.rho[cell] : (T)1;
  const T cx = rho * A.sx, cy = rho * A.sy, cz = rho * A.sz, cm = A.sm;

  // phase 1 (lane t = y): temporal mixing at the nodes and the x sweeps, one z row at a time
  T U[N][N], V[N][N];                                      // [z][x]
  {
    const T* xc = xs + ((size_t)(lcz * p) * nby + (lcy * p + t)) * nbx + lcx * p;
    const int k0 = act ? uptr_s[i] : 0, k1 = act ? uptr_s[i + 1] : 0;
#pragma unroll
    for (int z = 0; z < N; ++z) {
      T a[N], b[N];
#pragma unroll
      for (int x = 0; x < N; ++x) { a[x] = 0; b[x] = 0; }
      for (int k = k0; k < k1; ++k) {
        const T cmk = um_s[k], cnk = un_s[k];
        const T* r = xc + (size_t)ucol_s[k] * NB + z * nby * nbx;
#pragma unroll
        for (int x = 0; x < N; ++x) {
          const T v = r[x];
          a[x] += cmk * v;
          b[x] += cnk * v;
        }
      }
#pragma unroll
      for (int x = 0; x < N; ++x) {
        T u = 0, ka = 0, mb = 0;
#pragma unroll
        for (int q = 0; q < N; ++q) {
          u += SYM(A.M, x, q) * a[q];
          ka += SYM(A.K, x, q) * a[q];
          mb += SYM(A.M, x, q) * b[q];
        }
        U[z][x] = u;
        V[z][x] = cx * ka + cm * mb;
      }
    }
  }
  __syncthreads();                                         // every team has read its input

  // phase 2, one x slice at a time: z sweeps (lane t = y), exchange, y sweeps (lane t = z)
  T Y[N][N];                                               // [y][x] of plane z = t
  T* sc = scr + (size_t)(act ? team : 0) * 2 * N * N;
#pragma unroll
  for (int xx = 0; xx < N; ++xx) {
#pragma unroll
    for (int z = 0; z < N; ++z) {
      T w = 0, kz = 0, zz = 0;
#pragma unroll
      for (int q = 0; q < N; ++q) {
        w += SYM(A.M, z, q) * V[q][xx];
        kz += SYM(A.K, z, q) * U[q][xx];
        zz += SYM(A.M, z, q) * U[q][xx];
      }
      if (act) {
        sc[z * N + t] = w + cz * kz;
        sc[N * N + z * N + t] = zz;
      }
    }
    wave_sync_lds();
    T w2[N], z2[N];
#pragma unroll
    for (int yy = 0; yy < N; ++yy) {
      w2[yy] = act ? sc[t * N + yy] : (T)0;
      z2[yy] = act ? sc[N * N + t * N + yy] : (T)0;
    }
#pragma unroll
    for (int yy = 0; yy < N; ++yy) {
      T my = 0, ky = 0;
#pragma unroll
      for (int q = 0; q < N; ++q) {
        my += SYM(A.M, yy, q) * w2[q];
        ky += SYM(A.K, yy, q) * z2[q];
      }
      Y[yy][xx] = my + cy * ky;
    }
    wave_sync_lds();
  }

  __syncthreads();                                         // every team is done with its slices
  for (int e = tid; e < n_t * NB; e += nthr) xs[e] = (T)0;
  __syncthreads();

  // sum the cell results into the brick, one cell parity class per round (cells of a class share
  // no node, so each sum meets no other one and the order is fixed)
  const int par = (lcx & 1) | ((lcy & 1) << 1) | ((lcz & 1) << 2);
  T* o = xs + (size_t)i * NB + ((size_t)(lcz * p + t) * nby + lcy * p) * nbx + lcx * p;
  for (int r = 0; r < 8; ++r) {
    if (act && par == r) {
#pragma unroll
      for (int yy = 0; yy < N; ++yy)
#pragma unroll
        for (int xx = 0; xx < N; ++xx) {
          if constexpr (sizeof(T) == 8)    // one LDS add instruction (measured slower for FP32)
            __hip_atomic_fetch_add(o + yy * nbx + xx, Y[yy][xx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          else
            o[yy * nbx + xx] += Y[yy][xx];
        }
    }
    __syncthreads();
  }

  brick_write<T, OP_BATCH>(g, A.L, P, n_t, xs, zl, A.scale, A.overwrite, A.base, A.y);
}

template <class T, int N>
void launch_brick(const GeomDesc& g, const CartTables& ct, const TemporalDev<T>& tp, const T* x, T* y,
                  T scale, const T* base, bool overwrite, const BrickPlan& pl, hipStream_t s) {
  BrickOpArgs<T, N> A;
  for (int a = 0; a < N; ++a)
    for (int b = 0; b < N; ++b) {      // canonical representatives (see sym_row)
      const int r = sym_row<N>(a, b), c = sym_col<N>(a, b);
      A.M[a][b] = (T)ct.M[r * N + c];
      A.K[a][b] = (T)ct.K[r * N + c];
    }
  A.sx = (T)(g.h[1] * g.h[2] / g.h[0]);
  A.sy = (T)(g.h[0] * g.h[2] / g.h[1]);
  A.sz = (T)(g.h[0] * g.h[1] / g.h[2]);
  A.sm = (T)(g.h[0] * g.h[1] * g.h[2]);
  A.g = g;
  A.tp = tp;
  A.x = x;
  A.y = y;
  A.base = base;
  A.scale = scale;
  A.overwrite = overwrite ? 1 : 0;
  BrickLaunch L[8];
  brick_launches(g, pl, L);
  for (int colour = 0; colour < 8; ++colour) {
    if (L[colour].nblocks == 0) continue;
    A.L = L[colour];
    hipLaunchKernelGGL((st_apply3_brick<T, N>), dim3((unsigned)L[colour].nblocks), dim3(pl.waves * 64), pl.lds, s, A);
    STMG_CHECK_LAUNCH();
  }
}

}  // namespace

CartTables make_cart_tables(const LevelTables& lt) {
  const int n = lt.n;
  CartTables ct;
  ct.n = n;
  ct.M.assign((size_t)n * n, 0.0);
  ct.K.assign((size_t)n * n, 0.0);
  // nodal derivatives at the Gauss points: dphi[q][i] = sum_r D[q][r] S[r][i]
  std::vector<double> dphi((size_t)n * n, 0.0);
  for (int q = 0; q < n; ++q)
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int r = 0; r < n; ++r) s += lt.D[q * n + r] * lt.S[r * n + i];
      dphi[q * n + i] = s;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double m = 0.0, k = 0.0;
      for (int q = 0; q < n; ++q) {
        m += lt.gw[q] * lt.S[q * n + i] * lt.S[q * n + j];
        k += lt.gw[q] * dphi[q * n + i] * dphi[q * n + j];
      }
      ct.M[i * n + j] = m;
      ct.K[i * n + j] = k;
    }
  return ct;
}

bool brick_applicable(const GeomDesc& g) {
  return g.dim == 3 && !g.verts && !g.rho_q && g.n >= 2 && g.n <= MAXN;
}

template <class T>
void st_apply_brick(const GeomDesc& g, const CartTables& ct, const TemporalDev<T>& tp, const T* x, T* y,
                    T scale, hipStream_t s, const T* base, bool overwrite) {
  if (!brick_applicable(g)) fail(STMG_E_UNSUPPORTED, "the brick operator needs a 3D Cartesian level");
  if (g.ncells == 0 || tp.n_t == 0) return;
  if (!tp.uptr) fail(STMG_E_STATE, "temporal factors without their union pattern");
  const size_t csr = sizeof(T) * (size_t)(1 + 2 * tp.unnz) + sizeof(int) * (size_t)(tp.n_t + 1 + tp.unnz);
  BrickPlan pl;
  auto run = [&](auto tag, int vgprs) {
    constexpr int N = decltype(tag)::value;
    // long bricks measured faster in FP64 (lower degrees) and slower in FP32 (Q4: 16 x 1 x 1)
    if (!plan_brick(g, tp.n_t, tp.n_t, N, sizeof(T), 2 * N * N, csr, vgprs, pl, true, sizeof(T) == 8))
      fail(STMG_E_UNSUPPORTED, "no brick fits the temporal DoFs");
    launch_brick<T, N>(g, ct, tp, x, y, scale, base, overwrite, pl, s);
  };
  switch (g.n) {
    case 2: { static const int v = kernel_vgprs(st_apply3_brick<T, 2>); run(std::integral_constant<int, 2>(), v); break; }
    case 3: { static const int v = kernel_vgprs(st_apply3_brick<T, 3>); run(std::integral_constant<int, 3>(), v); break; }
    case 4: { static const int v = kernel_vgprs(st_apply3_brick<T, 4>); run(std::integral_constant<int, 4>(), v); break; }
    case 5: { static const int v = kernel_vgprs(st_apply3_brick<T, 5>); run(std::integral_constant<int, 5>(), v); break; }
    default: fail(STMG_E_UNSUPPORTED, "p must be 1..4");
  }
}

template void st_apply_brick<double>(const GeomDesc&, const CartTables&, const TemporalDev<double>&,
                                     const double*, double*, double, hipStream_t, const double*, bool);
template void st_apply_brick<float>(const GeomDesc&, const CartTables&, const TemporalDev<float>&,
                                    const float*, float*, float, hipStream_t, const float*, bool);

}  // namespace stmg
