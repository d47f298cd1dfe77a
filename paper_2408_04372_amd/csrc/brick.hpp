// Brick tiling shared by the brick operator and the brick smoother (Cartesian 3D levels).
//
// A workgroup owns a brick of B_x x B_y x B_z cells.  The brick's lattice nodes, (p B + 1) per
// direction and every temporal plane, are staged once in LDS; the cells' results are summed into
// that LDS copy in eight rounds, one per cell parity class (cells of one class share no node), and
// every node of the brick is then written to HBM once.  Bricks are launched in 2^3 parity colours:
// bricks of one colour share no node, and a node on a brick face is stored by the brick of the
// lowest colour holding it (with the base vector, in overwrite mode) and updated by the others in
// colour order.  The summation order is fixed (no two additions of a round meet at a node; in FP64
// they are single LDS add instructions), so results are bitwise reproducible, with no global atomics.
#pragma once

#include <algorithm>

#include "device.hpp"
#include "kernels.hpp"

namespace stmg {

// launch description of one brick colour
struct BrickLaunch {
  int B[3];           // brick size in cells
  int NBd[3];         // brick lattice nodes per direction (p B + 1)
  int nbt[3];         // bricks per direction (all colours)
  int nbc[3];         // bricks of this colour per direction
  int colour;
  int nblocks;
};

// this workgroup's brick
struct BrickPos {
  int b[3];           // brick coordinates
  int c0[3];          // first cell
  int nc[3];          // cells of the brick inside the mesh (the last brick per direction may be short)
  int g0[3];          // first lattice node
  int NB;             // nodes per temporal plane of the (full-size) brick box
};

__device__ inline BrickPos brick_pos(const BrickLaunch& L, const GeomDesc& g) {
  BrickPos P;
  const int lb = xcd_swizzle(blockIdx.x, L.nblocks);
  const int ib[3] = {lb % L.nbc[0], (lb / L.nbc[0]) % L.nbc[1], lb / (L.nbc[0] * L.nbc[1])};
  for (int d = 0; d < 3; ++d) {
    P.b[d] = 2 * ib[d] + ((L.colour >> d) & 1);
    P.c0[d] = P.b[d] * L.B[d];
    P.nc[d] = min(L.B[d], g.nc[d] - P.c0[d]);
    P.g0[d] = P.c0[d] * g.p;
  }
  P.NB = L.NBd[0] * L.NBd[1] * L.NBd[2];
  return P;
}

// Thread layout of the stage and write-back loops.  The brick's node box is a stack of
// NBd[2] * n_t planes (lz, j) of NBd[0] x NBd[1] nodes.  A thread keeps one (lx, ly) position of a
// plane (several when a plane has more nodes than the workgroup has threads) and walks the planes
// lz = slot, slot + step, ... with a carried (lz, j) counter, so the x and y parts of every index and
// predicate are formed once per thread and a plane step costs an add and a compare.  Planes come in
// batches of ROW_BATCH so that every global load of a batch is issued before the first of them is
// used (24 covers the 20 planes per thread of a Q4 brick one cell deep with four temporal DoFs).
struct PlaneWalk {
  int np;             // nodes per plane
  int e0, estep;      // first position of this thread and the step between its positions
  int slot, step;     // first lz and the lz step (step <= NBd[2])
  __device__ PlaneWalk(int tid, int nthr, const int NBd[3]) {
    np = NBd[0] * NBd[1];
    if (np <= nthr) {
      step = min(nthr / np, NBd[2]);
      slot = tid / np;
      e0 = slot < step ? tid - slot * np : np;    // threads past the last slot have no position
      estep = np;
    } else {
      step = 1;
      slot = 0;
      e0 = tid;
      estep = nthr;
    }
  }
};

// Order LDS accesses of one wave: the LDS executes a wave's operations in issue order, so a value
// written by one lane is visible to another lane of the same wave once the compiler keeps the
// write before the read (a team never straddles two waves).
__device__ inline void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Zeros in global memory, never written: the load of a lane that needs no value reads one (lanes of
// a wave reading one address cost one request).
static __device__ double brick_zero_f64 = 0.0;
static __device__ float brick_zero_f32 = 0.0f;
__device__ inline const double* brick_zero(const double*) { return &brick_zero_f64; }
__device__ inline const float* brick_zero(const float*) { return &brick_zero_f32; }

// The batches below are straight-line code: every lane issues every load of a batch, from the node's
// address or from a zero, so no value needs a select (or a branch) after its load returns.  With
// conditional loads the compiler puts each load in a branch of its own and waits for it there, and
// selects after the loads keep one lane mask per batch entry alive (more than the scalar registers
// hold).  Global and LDS offsets advance by additions along the (lz, j) walk.

// Batch size for a walk: entries past a position's last plane still cost a load, so a workgroup
// whose positions hold few planes (small bricks) takes a smaller batch (the choice is uniform).
__device__ inline int brick_batch(const PlaneWalk& w, const BrickLaunch& L, int n_t, int max_batch) {
  const int per = n_t * ((L.NBd[2] + w.step - 1) / w.step);   // (lz, j) planes of one position, at most
  return per <= 4 ? 4 : (per <= 8 || max_batch <= 8) ? 8 : max_batch;
}

template <class T, int ROW_BATCH>
__device__ inline void brick_stage_batch(const GeomDesc& g, const BrickLaunch& L, const BrickPos& P, int n_t,
                                         const T* __restrict__ x, T* xs, const PlaneWalk& w) {
  const int nbx = L.NBd[0], nbz = L.NBd[2];
  const int nn0 = g.nn[0], nn1 = g.nn[1], nn2 = g.nn[2];
  const long long nn01 = (long long)nn0 * nn1;
  const T* zero = brick_zero(x);
  const long long zstep = (long long)w.step * nn01, wrap = g.nx - (long long)nbz * nn01;
  const int sstep = w.step * w.np, swrap = P.NB - nbz * w.np;
  for (int e = w.e0; e < w.np; e += w.estep) {
    const int ly = e / nbx, lx = e - ly * nbx;
    const int gx = P.g0[0] + lx, gy = P.g0[1] + ly;
    const bool inxy = gx > 0 && gx < nn0 - 1 && gy > 0 && gy < nn1 - 1;
    T* sp = xs + e;
    int lz = w.slot, j = 0, so = lz * w.np;
    long long off = (long long)(P.g0[2] + lz) * nn01 + (long long)gy * nn0 + gx;
    while (j < n_t) {
      T v[ROW_BATCH];
      int dst[ROW_BATCH];         // -1: past the last plane
#pragma unroll
      for (int u = 0; u < ROW_BATCH; ++u) {
        const int gz = P.g0[2] + lz;
        const bool in = j < n_t && inxy && gz > 0 && gz < nn2 - 1;
        v[u] = *(in ? x + off : zero);
        dst[u] = j < n_t ? so : -1;
        lz += w.step;
        off += zstep;
        so += sstep;
        if (lz >= nbz) { lz -= nbz; ++j; off += wrap; so += swrap; }
      }
#pragma unroll
      for (int u = 0; u < ROW_BATCH; ++u)
        if (dst[u] >= 0) sp[dst[u]] = v[u];
    }
  }
}

// xs[j][node] = x on the brick's nodes for every temporal plane j < n_t (Dirichlet nodes and nodes
// past the lattice read as zero); batches of at most ROW_BATCH loads.
template <class T, int ROW_BATCH>
__device__ inline void brick_stage(const GeomDesc& g, const BrickLaunch& L, const BrickPos& P, int n_t,
                                   const T* __restrict__ x, T* xs) {
  const PlaneWalk w(threadIdx.x, blockDim.x, L.NBd);
  const int rb = brick_batch(w, L, n_t, ROW_BATCH);
  if (rb == 4) brick_stage_batch<T, 4>(g, L, P, n_t, x, xs, w);
  else if (rb == 8) brick_stage_batch<T, 8>(g, L, P, n_t, x, xs, w);
  else brick_stage_batch<T, ROW_BATCH>(g, L, P, n_t, x, xs, w);
}

template <class T, int ROW_BATCH>
__device__ inline void brick_write_batch(const GeomDesc& g, const BrickLaunch& L, const BrickPos& P, int n_t,
                                         const T* xs, const T* zl, T scale, int overwrite,
                                         const T* __restrict__ base, T* y, const PlaneWalk& w) {
  const int nbx = L.NBd[0], nbz = L.NBd[2];
  const int nn0 = g.nn[0], nn1 = g.nn[1], nn2 = g.nn[2];
  const long long nn01 = (long long)nn0 * nn1;
  const int p = g.p;
  const int last0 = P.nc[0] * p, last1 = P.nc[1] * p, last2 = P.nc[2] * p;
  const T* zero = brick_zero(xs);
  // a node on a shared brick face is stored by the brick of the lowest colour holding it
  const bool zlo_shared = P.b[2] > 0, zhi_shared = P.b[2] + 1 < L.nbt[2], zodd = (P.b[2] & 1) != 0;
  const long long zstep = (long long)w.step * nn01, wrap = g.nx - (long long)nbz * nn01;
  const int sstep = w.step * w.np, swrap = P.NB - nbz * w.np;
  for (int e = w.e0; e < w.np; e += w.estep) {
    const int ly = e / nbx, lx = e - ly * nbx;
    if (lx > last0 || ly > last1) continue;                     // outside the brick's cells
    const int gx = P.g0[0] + lx, gy = P.g0[1] + ly;
    const bool shx = (lx == 0 && P.b[0] > 0) || (lx == last0 && P.b[0] + 1 < L.nbt[0]);
    const bool shy = (ly == 0 && P.b[1] > 0) || (ly == last1 && P.b[1] + 1 < L.nbt[1]);
    const bool fxy = !(shx && (P.b[0] & 1)) && !(shy && (P.b[1] & 1));
    const bool bxy = gx == 0 || gx == nn0 - 1 || gy == 0 || gy == nn1 - 1;
    const T* sp = xs + e;
    int lz = w.slot, j = 0, so = lz * w.np;
    long long off = (long long)(P.g0[2] + lz) * nn01 + (long long)gy * nn0 + gx;
    while (j < n_t) {
      long long gi[ROW_BATCH];    // -1: no store
      T old[ROW_BATCH], v[ROW_BATCH];
#pragma unroll
      for (int u = 0; u < ROW_BATCH; ++u) {
        const bool ok = j < n_t && lz <= last2;
        const int gz = P.g0[2] + lz;
        const bool shz = (lz == 0 && zlo_shared) || (lz == last2 && zhi_shared);
        const bool store = overwrite && fxy && !(shz && zodd);
        const bool bnd = bxy || gz == 0 || gz == nn2 - 1;
        const bool upd = ok && !bnd && !store;                  // y += scale v
        const bool put = ok && store;                           // y = base + scale v (v = 0 on Dirichlet nodes)
        old[u] = *(upd ? y + off : ((put && base) ? base + off : zero));
        v[u] = *((ok && !bnd) ? sp + so : zl);
        gi[u] = (upd || put) ? off : -1;
        lz += w.step;
        off += zstep;
        so += sstep;
        if (lz >= nbz) { lz -= nbz; ++j; off += wrap; so += swrap; }
      }
#pragma unroll
      for (int u = 0; u < ROW_BATCH; ++u)
        if (gi[u] >= 0) y[gi[u]] = old[u] + scale * v[u];
    }
  }
}

// Write the brick's sums xs (n_t planes) to y:
//   overwrite: y = base + scale * xs by the brick of the lowest colour holding the node (base null:
//              zero), y += scale * xs by the others; Dirichlet nodes receive base (or zero) only;
//   otherwise: y += scale * xs on interior nodes.
// zl points to a zero in LDS; batches of at most ROW_BATCH loads.
template <class T, int ROW_BATCH>
__device__ inline void brick_write(const GeomDesc& g, const BrickLaunch& L, const BrickPos& P, int n_t,
                                   const T* xs, const T* zl, T scale, int overwrite, const T* __restrict__ base,
                                   T* y) {
  const PlaneWalk w(threadIdx.x, blockDim.x, L.NBd);
  const int rb = brick_batch(w, L, n_t, ROW_BATCH);
  if (rb == 4) brick_write_batch<T, 4>(g, L, P, n_t, xs, zl, scale, overwrite, base, y, w);
  else if (rb == 8) brick_write_batch<T, 8>(g, L, P, n_t, xs, zl, scale, overwrite, base, y, w);
  else brick_write_batch<T, ROW_BATCH>(g, L, P, n_t, xs, zl, scale, overwrite, base, y, w);
}


struct BrickPlan {
  int B[3] = {1, 1, 1};
  int waves = 1;
  size_t lds = 0;
};

// Registers of a kernel's waves (VGPRs), read once per instantiation; 128 when HIP cannot say.
template <class K>
inline int kernel_vgprs(K kernel) {
  hipFuncAttributes a;
  if (hipFuncGetAttributes(&a, reinterpret_cast<const void*>(kernel)) != hipSuccess || a.numRegs <= 0) {
    (void)hipGetLastError();
    return 128;
  }
  return a.numRegs;
}

// Brick size: the largest product of
//   - the share of owned nodes in the staged box (halo nodes are read twice),
//   - the share of a lattice row's bytes in the cache lines it touches (rows of NBd[0] nodes plus
//     about half a 128-byte line of neighbours' nodes),
//   - the lane use of the teams, and
//   - the occupancy: resident waves per CU (workgroups limited by LDS, 160 KB per CU, and by the
//     kernel's VGPRs, 512 per lane and SIMD) against 8, times 3/4 when only one workgroup fits a CU
//     (its staging, compute and write-back phases then run back to back),
// with at most 8 waves, every work item of the brick (items_per_cell per cell, one team of
// team_lanes lanes each, teams never straddling a wave) in one round of teams, and LDS (n_t planes
// of the box, team_scratch values per team, plus `extra` bytes; with scratch_in_box the team scratch
// reuses the box's planes and the larger of the two counts) within 72 KB.
inline bool plan_brick(const GeomDesc& g, int n_t, int items_per_cell, int team_lanes, size_t elem,
                       int team_scratch, size_t extra, int vgprs, BrickPlan& out, bool scratch_in_box = false,
                       bool long_bricks = false) {
  const int p = g.p;
  const int tpw = 64 / team_lanes;
  const int vg = std::max(8, (vgprs + 7) / 8 * 8);
  const int waves_simd = std::max(1, std::min(8, 512 / vg));
  static const int cand[][3] = {{4, 3, 2}, {4, 2, 2}, {3, 3, 2}, {3, 2, 2}, {2, 3, 2}, {2, 2, 2}, {6, 2, 1},
                                {4, 3, 1}, {4, 2, 1}, {3, 3, 1}, {3, 2, 1}, {2, 2, 1}, {2, 1, 1}, {1, 1, 1},
                                {6, 3, 2}, {8, 2, 2}, {16, 1, 1}};
  const int ncand = long_bricks ? 17 : 14;
  double best = -1.0;
  for (int ci = 0; ci < ncand; ++ci) {
    const int* c = cand[ci];
    int B[3] = {std::min(c[0], g.nc[0]), std::min(c[1], g.nc[1]), std::min(c[2], g.nc[2])};
    const long long items = (long long)B[0] * B[1] * B[2] * items_per_cell;
    const int waves = (int)((items + tpw - 1) / tpw);
    if (waves > 8) continue;
    const int nbd0 = p * B[0] + 1;
    const long long nb = (long long)nbd0 * (p * B[1] + 1) * (p * B[2] + 1);
    const size_t box = (size_t)n_t * nb, scr = (size_t)waves * tpw * team_scratch;
    const size_t lds = elem * (scratch_in_box ? std::max(box, scr) : box + scr) + extra;
    if (lds > 72 * 1024) continue;
    const double owned = (double)(p * B[0]) * (p * B[1]) * (p * B[2]) / (double)nb;
    const double row = (double)(nbd0 * elem) / (double)(nbd0 * elem + 64);
    const double use = (double)items / ((double)waves * tpw);
    const int simd_waves = (waves + 3) / 4;                    // waves of one workgroup per SIMD
    const int wgs = std::min((int)((160 * 1024) / lds), std::min(4 * waves_simd / waves, waves_simd / simd_waves));
    if (wgs < 1) continue;
    const double occ = std::min(1.0, (double)(wgs * waves) / 8.0) * (wgs >= 2 ? 1.0 : 0.75);
    const double score = owned * row * use * occ;
    if (score > best + 1e-9) {
      best = score;
      out.B[0] = B[0]; out.B[1] = B[1]; out.B[2] = B[2];
      out.waves = waves;
      out.lds = lds;
    }
  }
  return best > 0.0;
}

// per-colour launch descriptions; a colour without bricks has nblocks = 0
inline void brick_launches(const GeomDesc& g, const BrickPlan& pl, BrickLaunch out[8]) {
  for (int colour = 0; colour < 8; ++colour) {
    BrickLaunch& L = out[colour];
    long long cnt = 1;
    for (int d = 0; d < 3; ++d) {
      L.B[d] = pl.B[d];
      L.NBd[d] = g.p * pl.B[d] + 1;
      L.nbt[d] = (g.nc[d] + pl.B[d] - 1) / pl.B[d];
      const int o = (colour >> d) & 1;
      L.nbc[d] = (L.nbt[d] - o + 1) / 2;
      cnt *= L.nbc[d];
    }
    if (cnt > (1LL << 31) - 1) fail(STMG_E_UNSUPPORTED, "too many bricks");
    L.colour = colour;
    L.nblocks = (int)cnt;
  }
}

}  // namespace stmg
