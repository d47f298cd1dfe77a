// Level hierarchy, smoother set-up, relaxation estimates and the V-cycle
// (Section 3: Alg. stmg and Alg. mg-sequence).
//
// Level sequence (finest first): halve p while p > min_p, then halve the cell
// count per direction while every direction stays even and does not drop below
// coarse_cells; with time_mg, then lower the temporal degree k by one per level
// to its minimum and halve the number of time cells while it is even, all on the
// coarsest spatial mesh.  Coarse h-levels take the even-index vertex subset and
// re-discretise; their coefficient at a quadrature point is that of the finest
// descendant cell whose reference sub-box contains the point.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>

#include "handle.hpp"

namespace stmg {

template <> LevelData<double>& ldata<double>(Level& L) { return L.d64; }
template <> LevelData<float>& ldata<float>(Level& L) { return L.d32; }
template <> const TemporalDev<double>& tdev<double>(const Level& L) { return L.ts->tp64.dev; }
template <> const TemporalDev<float>& tdev<float>(const Level& L) { return L.ts->tp32.dev; }

// ------------------------------------------------------------------ timer
void Timer::mark(int t, hipStream_t s) {
  if (!on) return;
  if (used == ev.size()) {
    hipEvent_t e;
    STMG_HIP(hipEventCreate(&e));
    ev.push_back(e);
    tag.push_back(0);
  }
  tag[used] = t;
  STMG_HIP(hipEventRecord(ev[used], s));
  ++used;
}
void Timer::accumulate(double out[4]) {
  if (used < 2) return;
  STMG_HIP(hipEventSynchronize(ev[used - 1]));
  for (size_t i = 0; i + 1 < used; ++i) {
    float ms = 0.f;
    STMG_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
    out[tag[i]] += ms * 1e-3;
  }
}
Timer::~Timer() {
  for (auto e : ev) (void)hipEventDestroy(e);
}

void KernelTimer::begin(int k, hipStream_t s) {
  if (!on) return;
  if (2 * used + 2 > ev.size()) {
    for (int i = 0; i < 2; ++i) {
      hipEvent_t e;
      STMG_HIP(hipEventCreate(&e));
      ev.push_back(e);
    }
    kind.push_back(0);
  }
  kind[used] = k;
  STMG_HIP(hipEventRecord(ev[2 * used], s));
}
void KernelTimer::end(hipStream_t s) {
  if (!on) return;
  STMG_HIP(hipEventRecord(ev[2 * used + 1], s));
  ++used;
  if (used >= 4096) flush();
}
void KernelTimer::flush() {
  if (used == 0) return;
  STMG_HIP(hipEventSynchronize(ev[2 * used - 1]));
  for (size_t i = 0; i < used; ++i) {
    float ms = 0.f;
    STMG_HIP(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
    n[kind[i]] += 1;
    t[kind[i]] += ms * 1e-3;
  }
  used = 0;
}
KernelTimer::~KernelTimer() {
  for (auto e : ev) (void)hipEventDestroy(e);
}

// ------------------------------------------------------------------ 1D tables
LevelTables make_level_tables(int p) {
  LevelTables t;
  int n = p + 1;
  t.n = n;
  hm::Vec gq, gw;
  hm::gauss(n, gq, gw);
  hm::Vec nodes = hm::gauss_lobatto(n);
  hm::Mat V, D, Vg, Dg;
  hm::lagrange(nodes, gq, V, D);      // GLL basis at Gauss points
  hm::lagrange(gq, gq, Vg, Dg);       // Gauss-point Lagrange basis: collocation derivative
  t.S.assign(V.a.begin(), V.a.end());
  t.D.assign(Dg.a.begin(), Dg.a.end());
  t.gq = gq;
  t.gw = gw;
  return t;
}

namespace {

}  // namespace

// CSR of the nonzeros of a dense n x n matrix; returns the number of nonzeros
template <class T>
int upload_csr(const hm::Mat& A, DevBuf& ptr, DevBuf& col, DevBuf& val, hipStream_t s) {
  std::vector<int> p{0}, c;
  std::vector<T> v;
  for (int i = 0; i < A.r; ++i) {
    for (int j = 0; j < A.c; ++j)
      if (A(i, j) != 0.0) { c.push_back(j); v.push_back((T)A(i, j)); }
    p.push_back((int)c.size());
  }
  const int nnz = (int)c.size();
  if (c.empty()) { c.push_back(0); v.push_back(0); }
  ptr = upload(p, s);
  col = upload(c, s);
  val = upload(v, s);
  return nnz;
}

template int upload_csr<double>(const hm::Mat&, DevBuf&, DevBuf&, DevBuf&, hipStream_t);
template int upload_csr<float>(const hm::Mat&, DevBuf&, DevBuf&, DevBuf&, hipStream_t);

namespace {

template <class T>
void make_temporal(const hm::Temporal& tm, TemporalBufs<T>& tb, hipStream_t s) {
  tb.dev.mnnz = upload_csr<T>(tm.M_T, tb.mptr, tb.mcol, tb.mval, s);
  tb.dev.nnnz = upload_csr<T>(tm.N_T, tb.nptr, tb.ncol, tb.nval, s);
  tb.dev.n_t = tm.n_t;
  tb.dev.mptr = tb.mptr.template as<int>(); tb.dev.mcol = tb.mcol.template as<int>(); tb.dev.mval = tb.mval.template as<T>();
  tb.dev.nptr = tb.nptr.template as<int>(); tb.dev.ncol = tb.ncol.template as<int>(); tb.dev.nval = tb.nval.template as<T>();
  std::vector<int> up{0}, uc;
  std::vector<T> um, un;
  for (int i = 0; i < tm.n_t; ++i) {
    for (int j = 0; j < tm.n_t; ++j)
      if (tm.M_T(i, j) != 0.0 || tm.N_T(i, j) != 0.0) {
        uc.push_back(j);
        um.push_back((T)tm.M_T(i, j));
        un.push_back((T)tm.N_T(i, j));
      }
    up.push_back((int)uc.size());
  }
  tb.dev.unnz = (int)uc.size();
  if (uc.empty()) { uc.push_back(0); um.push_back(0); un.push_back(0); }
  tb.uptr = upload(up, s);
  tb.ucol = upload(uc, s);
  tb.umval = upload(um, s);
  tb.unval = upload(un, s);
  tb.dev.uptr = tb.uptr.template as<int>(); tb.dev.ucol = tb.ucol.template as<int>();
  tb.dev.umval = tb.umval.template as<T>(); tb.dev.unval = tb.unval.template as<T>();
}

}  // namespace

// 1D prolongation from a coarse (pc, ncc cells) to a fine (pf, ncf cells) lattice along one axis
// The transfers act on interior nodes only (P_full = M_f P M_c with the interior indicators
// M); the indicator of a tensor lattice is the product of per-axis indicators, so it is
// folded into the 1D factors: first and last rows and columns are dropped.
std::vector<std::vector<std::pair<int, double>>> transfer_1d_rows(int pc, int ncc, int pf, int ncf) {
  int r = ncf / ncc;
  int Nf = pf * ncf + 1, Nc = pc * ncc + 1;
  hm::Vec fn = hm::gauss_lobatto(pf + 1), cn = hm::gauss_lobatto(pc + 1);
  std::vector<std::vector<std::pair<int, double>>> rows(Nf);
  for (int g = 0; g < Nf; ++g) {
    int cf = std::min(g / pf, ncf - 1);
    int lf = g - cf * pf;
    int cc = cf / r;
    double xi = ((cf - cc * r) + fn[lf]) / r;
    hm::Mat V, D;
    hm::lagrange(cn, hm::Vec{xi}, V, D);
    if (g == 0 || g == Nf - 1) continue;                 // Dirichlet fine node
    for (int j = 0; j <= pc; ++j) {
      double w = V(0, j);
      if (std::fabs(w) < 1e-14) continue;
      const int c = cc * pc + j;
      if (c == 0 || c == Nc - 1) continue;                // Dirichlet coarse node
      rows[g].push_back({cc * pc + j, w});
    }
  }
  return rows;
}

namespace {

void transfer_1d(int pc, int ncc, int pf, int ncf, Transfer1D& P, Transfer1D& R, hipStream_t s) {
  const std::vector<std::vector<std::pair<int, double>>> rows = transfer_1d_rows(pc, ncc, pf, ncf);
  // R = P^T, each column's entries in increasing fine index
  std::vector<std::vector<std::pair<int, double>>> cols(pc * ncc + 1);
  for (int g = 0; g < (int)rows.size(); ++g)
    for (auto& e : rows[g]) cols[e.first].push_back({g, e.second});
  auto up = [&](const std::vector<std::vector<std::pair<int, double>>>& L, Transfer1D& T) {
    std::vector<int> ptr{0}, col;
    std::vector<double> w;
    std::vector<float> wf;
    T.max_row = 0;
    for (auto& row : L) {
      for (auto& e : row) { col.push_back(e.first); w.push_back(e.second); wf.push_back((float)e.second); }
      ptr.push_back((int)col.size());
      T.max_row = std::max(T.max_row, (int)row.size());
    }
    T.len_out = (int)L.size();
    T.nnz = (int)col.size();
    T.ptr_h = ptr;
    T.col_h = col;
    T.w_h = w;
    T.ptr = upload(ptr, s);
    T.col = upload(col, s);
    T.w64 = upload(w, s);
    T.w32 = upload(wf, s);
  };
  up(rows, P);
  up(cols, R);
}

// Per-tile input range of a banded 1D factor: lo[t], hi[t] over the rows of tile t (tiles of
// `tile` consecutive output rows; lo > hi when every row of the tile is empty).
void tile_ranges(const Transfer1D& A, int tile, std::vector<int>& lo, std::vector<int>& hi) {
  const int nt = (A.len_out + tile - 1) / tile;
  lo.assign(nt, 0);
  hi.assign(nt, -1);
  for (int t = 0; t < nt; ++t) {
    int l = 1 << 30, h = -1;
    for (int r = t * tile; r < std::min(A.len_out, (t + 1) * tile); ++r) {
      const int k0 = A.ptr_h[r], k1 = A.ptr_h[r + 1];
      if (k1 > k0) { l = std::min(l, A.col_h[k0]); h = std::max(h, A.col_h[k1 - 1]); }
    }
    if (h >= l) { lo[t] = l; hi[t] = h; }
  }
}

// Tiles and tables of the fused 3D transfer with factors A[3] (see Tensor3Plan): the x-y tile
// with the most output nodes per workgroup (up to 256), ties broken by a smaller input patch per
// output (by at least 10 %, else the longer x rows), with the patch within 2048 nodes; z chunks of 16 planes (4 on short axes).  Not ok when
// an x or y row is longer than 10 entries (R of an h-transfer at p >= 3) or no tile fits.
void build_fused3(const std::array<Transfer1D, 3>& A, Fused3& F, hipStream_t s) {
  Tensor3Plan& best = F.pl;
  best = Tensor3Plan();
  int kmax = 2;
  for (int d = 0; d < 2; ++d) kmax = std::max(kmax, A[d].max_row);
  static const int ks[] = {2, 3, 4, 5, 6, 8, 10};
  int kp = 0;
  for (int k : ks)
    if (k >= kmax) { kp = k; break; }
  if (kp == 0) return;                      // rows too long: 1D sweeps instead
  auto span = [&](int d, int tile) {
    std::vector<int> lo, hi;
    tile_ranges(A[d], tile, lo, hi);
    int m = 1;
    for (size_t i = 0; i < lo.size(); ++i) m = std::max(m, hi[i] - lo[i] + 1);
    return m;
  };
  static const int cand[][2] = {{64, 4}, {32, 8}, {16, 16}, {64, 2}, {32, 4}, {16, 8}, {8, 8}, {64, 1}, {32, 2},
                                {16, 4}, {8, 4}, {4, 4}, {16, 2}, {8, 2}, {4, 2}, {2, 2}, {8, 1}, {4, 1}, {2, 1}, {1, 1}};
  long long bestn = 0;
  double bestr = 0.0;
  for (auto& c : cand) {
    int cap0 = 1, cap1 = 1;
    while (cap0 < A[0].len_out) cap0 *= 2;
    while (cap1 < A[1].len_out) cap1 *= 2;
    if (c[0] > cap0 || c[1] > cap1) continue;
    const int S0 = span(0, c[0]), S1 = span(1, c[1]);
    if ((long long)S0 * S1 > 2048) continue;
    const long long n = (long long)c[0] * c[1];
    const double r = (double)S0 * S1 / (double)n;
    if (n > bestn || (n == bestn && r < 0.9 * bestr)) {      // longer x rows unless 10 % fewer reads
      bestn = n;
      bestr = r;
      best.T[0] = c[0]; best.T[1] = c[1];
      best.S[0] = S0; best.S[1] = S1;
    }
  }
  if (bestn == 0) return;
  best.T[2] = A[2].len_out >= 32 ? 16 : 4;
  best.S[2] = span(2, best.T[2]);
  best.kmax = kp;
  while ((1 << best.lg[0]) < best.T[0]) ++best.lg[0];
  std::vector<int> lo, hi;
  for (int d = 0; d < 3; ++d) {
    tile_ranges(A[d], best.T[d], lo, hi);
    best.nt[d] = (int)lo.size();
    std::vector<int> col;
    std::vector<double> w;
    if (d < 2) {
      col.assign((size_t)A[d].len_out * kp, 0);
      w.assign((size_t)A[d].len_out * kp, 0.0);
      for (int r = 0; r < A[d].len_out; ++r) {
        const int t = r / best.T[d];
        for (int k = A[d].ptr_h[r], q = 0; k < A[d].ptr_h[r + 1]; ++k, ++q) {
          col[(size_t)r * kp + q] = A[d].col_h[k] - lo[t];
          w[(size_t)r * kp + q] = A[d].w_h[k];
        }
      }
    } else {
      // dense weights of each chunk: w[chunk][k][j] multiplies input plane lo[chunk] + j
      const int TZ = best.T[2], SZ = best.S[2];
      w.assign((size_t)best.nt[2] * TZ * SZ, 0.0);
      for (int r = 0; r < A[d].len_out; ++r) {
        const int t = r / TZ, k0 = r - t * TZ;
        for (int k = A[d].ptr_h[r]; k < A[d].ptr_h[r + 1]; ++k)
          w[((size_t)t * TZ + k0) * SZ + (A[d].col_h[k] - lo[t])] = A[d].w_h[k];
      }
    }
    std::vector<float> wf(w.begin(), w.end());
    F.lo[d] = upload(lo, s);
    F.hi[d] = upload(hi, s);
    if (!col.empty()) F.col[d] = upload(col, s);
    F.w64[d] = upload(w, s);
    F.w32[d] = upload(wf, s);
  }
  best.ok = true;
}

void init_geom(Level& L, int dim, const stmg_config& cfg) {
  GeomDesc& g = L.g;
  g.dim = dim;
  g.p = L.p;
  g.n = L.p + 1;
  g.nx = 1;
  g.ncells = 1;
  for (int d = 0; d < 3; ++d) {
    g.nc[d] = d < dim ? L.cells[d] : 1;
    g.nn[d] = d < dim ? L.p * L.cells[d] + 1 : 1;
    g.nx *= g.nn[d];
    g.ncells *= g.nc[d];
    g.lo[d] = cfg.lo[d];
    g.h[d] = d < dim ? (cfg.hi[d] - cfg.lo[d]) / L.cells[d] : 1.0;
  }
}

void boundary_lists(Level& L, hipStream_t s) {
  const GeomDesc& g = L.g;
  std::vector<int> b;
  std::vector<unsigned char> m(g.nx);
  for (long long z = 0; z < g.nn[2]; ++z)
    for (long long y = 0; y < g.nn[1]; ++y)
      for (long long x = 0; x < g.nn[0]; ++x) {
        long long idx = (z * g.nn[1] + y) * g.nn[0] + x;
        bool bd = x == 0 || x == g.nn[0] - 1 || y == 0 || y == g.nn[1] - 1 ||
                  (g.dim == 3 && (z == 0 || z == g.nn[2] - 1));
        m[idx] = bd ? 0 : 1;
        if (bd) b.push_back((int)idx);
      }
  L.nb = (long long)b.size();
  L.n_int = g.nx - L.nb;
  L.bidx = upload(b, s);
  L.mask = upload(m, s);
}

// coefficient data of a level: per cell on the finest mesh, per quadrature point on coarse h-levels
void level_coefficients(Level& L, const std::vector<double>& coef_fine, const int fine_cells[3],
                        hipStream_t s) {
  const GeomDesc& g = L.g;
  if (L.ratio == 1) {
    L.rho = upload(coef_fine, s);
    L.g.rho_q = 0;
  } else {
    int n = g.n;
    int nq = g.dim == 3 ? n * n * n : n * n;
    std::vector<double> rq((size_t)g.ncells * nq);
    for (long long c = 0; c < g.ncells; ++c) {
      long long cx = c % g.nc[0], cy = (c / g.nc[0]) % g.nc[1], cz = c / ((long long)g.nc[0] * g.nc[1]);
      for (int q = 0; q < nq; ++q) {
        int qi[3] = {q % n, (q / n) % n, q / (n * n)};
        long long fc[3] = {cx, cy, cz};
        for (int d = 0; d < g.dim; ++d) {
          long long sub = (long long)std::floor(L.lt.gq[qi[d]] * L.ratio);
          if (sub > L.ratio - 1) sub = L.ratio - 1;
          fc[d] = fc[d] * L.ratio + sub;
        }
        long long fidx = fc[0] + (long long)fine_cells[0] * (fc[1] + (g.dim == 3 ? (long long)fine_cells[1] * fc[2] : 0));
        rq[(size_t)c * nq + q] = coef_fine[fidx];
      }
    }
    L.rho = upload(rq, s);
    L.g.rho_q = 1;
  }
  L.g.rho = L.rho.as<double>();
}

// principal blocks A_KK, M_KK by probing the matrix-free operator, then the generalised
// eigenproblem A Q = M Q Lambda (rocSOLVER, batched) and the per-mode temporal inverses
// separable smoother: per-axis 1D tables for the four boundary cases, cell-mean coefficient
template <class T> static void upload_fdm(LevelData<T>& d, const std::vector<double>& q, const std::vector<double>& lam,
                                          const std::vector<double>& rho, const std::vector<double>& tmat,
                                          hipStream_t s) {
  auto cv = [](const std::vector<double>& v) { return std::vector<T>(v.begin(), v.end()); };
  d.fq = upload(cv(q), s);
  d.fl = upload(cv(lam), s);
  d.frho = upload(cv(rho), s);
  d.ftm = upload(cv(tmat), s);
}

void setup_fdm(stmg_handle* h, Level& L) {
  hipStream_t s = h->stream;
  const int n = L.g.n, p = L.g.p, dim = L.g.dim;
  hm::Vec xq, wq;
  hm::gauss(n, xq, wq);
  hm::Mat V, D;
  hm::lagrange(hm::gauss_lobatto(n), xq, V, D);
  std::vector<double> q((size_t)3 * 4 * n * n, 0.0), lam((size_t)3 * 4 * n, 0.0);
  for (int a = 0; a < dim; ++a) {
    const double hx = (h->cfg.hi[a] - h->cfg.lo[a]) / L.cells[a];
    hm::Mat Me(n, n), Ae(n, n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double m = 0.0, k = 0.0;
        for (int t = 0; t < n; ++t) {
          m += wq[t] * V(t, i) * V(t, j);
          k += wq[t] * D(t, i) * D(t, j);
        }
        Me(i, j) = hx * m;
        Ae(i, j) = k / hx;
      }
    for (int bc = 0; bc < 4; ++bc) {
      const bool lower = bc & 1, upper = bc & 2;
      hm::Mat M1 = Me, A1 = Ae;
      if (!lower) { M1(0, 0) += Me(p, p); A1(0, 0) += Ae(p, p); }
      if (!upper) { M1(p, p) += Me(0, 0); A1(p, p) += Ae(0, 0); }
      for (int e : {0, p}) {
        if ((e == 0 && !lower) || (e == p && !upper)) continue;
        for (int i = 0; i < n; ++i) { M1(e, i) = M1(i, e) = 0.0; A1(e, i) = A1(i, e) = 0.0; }
        M1(e, e) = 1.0;
        A1(e, e) = 1.0;
      }
      hm::Mat Q;
      hm::Vec lm;
      hm::sym_gen_eig(A1, M1, Q, lm);
      for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) q[(((size_t)a * 4 + bc) * n + r) * n + c] = Q(r, c);
      for (int c = 0; c < n; ++c) lam[((size_t)a * 4 + bc) * n + c] = lm[c];
    }
  }
  std::vector<double> tmat(L.ts->tm.M_tau.a);
  tmat.insert(tmat.end(), L.ts->tm.N_tilde.a.begin(), L.ts->tm.N_tilde.a.end());
  if (L.has64) upload_fdm<double>(L.d64, q, lam, L.rho_mean, tmat, s);
  if (L.has32) upload_fdm<float>(L.d32, q, lam, L.rho_mean, tmat, s);
}

// Vertex-patch smoother: per axis the assembled 1D matrices of two cells restricted to their
// 2p - 1 inner nodes, with generalised eigenpairs A Q = M Q diag(lambda), Q^T M Q = I.
void setup_patch(stmg_handle* h, Level& L) {
  hipStream_t s = h->stream;
  const int n = L.g.n, p = L.g.p, dim = L.g.dim, P = 2 * p - 1;
  hm::Vec xq, wq;
  hm::gauss(n, xq, wq);
  hm::Mat V, D;
  hm::lagrange(hm::gauss_lobatto(n), xq, V, D);
  std::vector<double> q((size_t)3 * P * P, 0.0), lam((size_t)3 * P, 0.0);
  for (int a = 0; a < dim; ++a) {
    const double hx = (h->cfg.hi[a] - h->cfg.lo[a]) / L.cells[a];
    hm::Mat M2(2 * p + 1, 2 * p + 1), A2(2 * p + 1, 2 * p + 1);
    for (int e = 0; e < 2; ++e)
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          double m = 0.0, k = 0.0;
          for (int t = 0; t < n; ++t) {
            m += wq[t] * V(t, i) * V(t, j);
            k += wq[t] * D(t, i) * D(t, j);
          }
          M2(e * p + i, e * p + j) += hx * m;
          A2(e * p + i, e * p + j) += k / hx;
        }
    hm::Mat M1(P, P), A1(P, P);
    for (int i = 0; i < P; ++i)
      for (int j = 0; j < P; ++j) {
        M1(i, j) = M2(i + 1, j + 1);
        A1(i, j) = A2(i + 1, j + 1);
      }
    hm::Mat Q;
    hm::Vec lm;
    hm::sym_gen_eig(A1, M1, Q, lm);
    for (int r = 0; r < P; ++r)
      for (int c = 0; c < P; ++c) q[((size_t)a * P + r) * P + c] = Q(r, c);
    for (int c = 0; c < P; ++c) lam[(size_t)a * P + c] = lm[c];
  }
  std::vector<double> tmat(L.ts->tm.M_tau.a);
  tmat.insert(tmat.end(), L.ts->tm.N_tilde.a.begin(), L.ts->tm.N_tilde.a.end());
  if (L.has64) upload_fdm<double>(L.d64, q, lam, L.rho_patch, tmat, s);
  if (L.has32) upload_fdm<float>(L.d32, q, lam, L.rho_patch, tmat, s);
}

namespace {

// Check of the generalised eigenpairs of a batch of cells (column-major ns x ns blocks):
// R = Q^T M Q must be the identity and AQ = A Q must equal T Lambda with T = M Q, column by
// column relative to max|AQ(:, k)| + |lambda_k| max|T(:, k)|.  flag[c] = 1 for a cell that fails
// either test or holds a non-finite value.  One workgroup per cell.
__global__ __launch_bounds__(128) void k_eig_check(int ns, const double* __restrict__ R,
                                                   const double* __restrict__ AQ, const double* __restrict__ T,
                                                   const double* __restrict__ lam, double tol, int* flag) {
  const long long c = blockIdx.x;
  const size_t off = (size_t)c * ns * ns;
  int bad = 0;
  for (int k = threadIdx.x; k < ns; k += blockDim.x) {
    const double lk = lam[c * ns + k];
    double orth = 0, an = 0, tn = 0, rr = 0;
    for (int i = 0; i < ns; ++i) {
      const size_t e = off + (size_t)k * ns + i;
      orth = fmax(orth, fabs(R[e] - (i == k ? 1.0 : 0.0)));
      an = fmax(an, fabs(AQ[e]));
      tn = fmax(tn, fabs(T[e]));
      rr = fmax(rr, fabs(AQ[e] - lk * T[e]));
    }
    // written so that a NaN anywhere fails
    if (!(orth <= tol) || !(rr <= tol * (an + fabs(lk) * tn)) || !(fabs(lk) < 1e300)) bad = 1;
  }
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) flag[c] = bad;
}

}  // namespace

void asm_eig_check(long long ncells, int ns, const double* R, const double* AQ, const double* T,
                   const double* lam, double tol, int* flag, hipStream_t s) {
  if (ncells <= 0) return;
  hipLaunchKernelGGL(k_eig_check, dim3((unsigned)ncells), dim3(128), 0, s, ns, R, AQ, T, lam, tol, flag);
  STMG_CHECK_LAUNCH();
}

// Bound on max|Q^T M Q - I| and on the relative eigen-residual of each local eigenpair; a
// converged FP64 solve of these blocks reaches about 1e-13 on both.
constexpr double EIG_CHECK_TOL = 1e-8;

void setup_smoother(stmg_handle* h, Level& L) {
  if (h->cfg.asm_variant == 1) {
    setup_fdm(h, L);
    return;
  }
  if (h->cfg.asm_variant == 2) {
    if (!patch_applicable(L.g, L.ts->tm.nt_cell))
      fail(STMG_E_UNSUPPORTED, "the vertex-patch smoother needs Cartesian levels with at least two cells per direction");
    setup_patch(h, L);
    return;
  }
  hipStream_t s = h->stream;
  const GeomDesc& g = L.g;
  const int ns = g.dim == 3 ? g.n * g.n * g.n : g.n * g.n;
  const long long nblk = g.ncells * ns * ns;
  DevBuf A(sizeof(double) * nblk), M(sizeof(double) * nblk);
  DevBuf x2(sizeof(double) * 2 * g.nx), y2(sizeof(double) * 2 * g.nx);
  // two-plane operator: plane 0 -> A_h x, plane 1 -> M_h x
  hm::Mat Mp(2, 2), Np(2, 2);
  Mp(0, 0) = 1.0;
  Np(1, 1) = 1.0;
  DevBuf mp, mc, mv, np_, nc, nv;
  TemporalDev<double> tp2;
  tp2.mnnz = upload_csr<double>(Mp, mp, mc, mv, s);
  tp2.nnnz = upload_csr<double>(Np, np_, nc, nv, s);
  tp2.n_t = 2;
  tp2.mptr = mp.as<int>(); tp2.mcol = mc.as<int>(); tp2.mval = mv.as<double>();
  tp2.nptr = np_.as<int>(); tp2.ncol = nc.as<int>(); tp2.nval = nv.as<double>();
  const int ncol = g.dim == 3 ? 27 : 9;
  // the probes run on the per-cell buffer path when a buffer of two planes is at hand (the
  // level's FP64 buffer, else a temporary one): one launch over all cells, and the gather writes
  // every node of y2; otherwise y2 is cleared and the colour path adds to it
  DevBuf pcb_tmp;
  double* pcb = L.n_t() >= 2 ? L.d64.cellbuf.as<double>() : nullptr;
  if (!pcb && pcb_tmp.try_alloc(sizeof(double) * (size_t)g.ncells * 2 * ns)) pcb = pcb_tmp.as<double>();
  fill<double>(x2.as<double>(), 0.0, 2 * g.nx, s);
  for (int colour = 0; colour < ncol; ++colour)
    for (int b = 0; b < ns; ++b) {
      asm_probe_set(g, colour, b, 1.0, x2.as<double>(), s);
      if (pcb) {
        st_apply<double>(g, L.lt, tp2, x2.as<double>(), y2.as<double>(), 1.0, s, pcb, nullptr, true);
      } else {
        fill<double>(y2.as<double>(), 0.0, 2 * g.nx, s);
        st_apply<double>(g, L.lt, tp2, x2.as<double>(), y2.as<double>(), 1.0, s);
      }
      asm_extract(g, colour, b, y2.as<double>(), A.as<double>(), M.as<double>(), s);
      asm_probe_set(g, colour, b, 0.0, x2.as<double>(), s);
    }
  pcb_tmp.release();
  x2.release();
  y2.release();
  DevBuf lam(sizeof(double) * g.ncells * ns), info(sizeof(int) * g.ncells);
  rocblas_handle rb;
  if (rocblas_create_handle(&rb) != rocblas_status_success) fail(STMG_E_HIP, "rocblas_create_handle failed");
  struct RbGuard {
    rocblas_handle h;
    ~RbGuard() { rocblas_destroy_handle(h); }
  } rb_guard{rb};
  rocblas_set_stream(rb, s);
  // Jacobi-based batched solver: the many small problems of one level are solved in one
  // pass each sweep (the tridiagonal route spends most of its time forming eigenvectors); the
  // reduction to standard form uses batched Cholesky and triangular solves, which are much
  // faster on these batches than the generalised solver's own column-by-column reduction.
  // Every cell's result is checked against copies of its blocks (M-orthonormality and the
  // eigen-residual); the batched generalised solver was seen to return, rarely and for a single
  // cell, a result off in the sixth digit from bitwise-identical input, so a failed check solves
  // the batch again from the copies (at most three solves, then the set-up fails).
  const size_t bb = sizeof(double) * (size_t)nblk;
  DevBuf A0(bb), M0(bb);
  STMG_HIP(hipMemcpyAsync(A0.get(), A.get(), bb, hipMemcpyDeviceToDevice, s));
  STMG_HIP(hipMemcpyAsync(M0.get(), M.get(), bb, hipMemcpyDeviceToDevice, s));
  DevBuf resid(sizeof(double) * g.ncells), sweeps(sizeof(int) * g.ncells), flag(sizeof(int) * g.ncells);
  const long long chunk = std::min<long long>(g.ncells, 4096);
  const size_t cb = sizeof(double) * (size_t)chunk * ns * ns;
  DevBuf Tb(cb), Rb(cb), AQb(cb);
  const double one = 1.0, zero = 0.0;
  const rocblas_stride bs = (rocblas_stride)ns * ns;
  long long nbad = 0, bad_cell = -1;
  for (int attempt = 0; attempt < 3; ++attempt) {
    if (attempt > 0) {
      STMG_HIP(hipMemcpyAsync(A.get(), A0.get(), bb, hipMemcpyDeviceToDevice, s));
      STMG_HIP(hipMemcpyAsync(M.get(), M0.get(), bb, hipMemcpyDeviceToDevice, s));
      ++h->eig_resolves;
    }
    // M = U^T U; C = U^{-T} A U^{-1} (two batched triangular solves, in place in A); C V = V Lambda
    // by the batched Jacobi solver; Q = U^{-1} V, so that A Q = M Q Lambda and Q^T M Q = I
    const int nc = (int)g.ncells;
    bad_cell = -1;
    if (rocsolver_dpotrf_strided_batched(rb, rocblas_fill_upper, ns, M.as<double>(), ns, bs, info.as<int>(), nc) !=
        rocblas_status_success)
      fail(STMG_E_HIP, "rocsolver_dpotrf_strided_batched failed");
    std::vector<int> inf = download<int>(info.get(), g.ncells, s);
    for (long long c = 0; c < g.ncells && bad_cell < 0; ++c)
      if (inf[c] != 0) bad_cell = c;
    if (bad_cell < 0) {
      rocblas_status t1 = rocblas_dtrsm_strided_batched(rb, rocblas_side_left, rocblas_fill_upper, rocblas_operation_transpose,
                                                        rocblas_diagonal_non_unit, ns, ns, &one, M.as<double>(), ns, bs,
                                                        A.as<double>(), ns, bs, nc);
      rocblas_status t2 = rocblas_dtrsm_strided_batched(rb, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                                                        rocblas_diagonal_non_unit, ns, ns, &one, M.as<double>(), ns, bs,
                                                        A.as<double>(), ns, bs, nc);
      rocblas_status ev = rocsolver_dsyevj_strided_batched(rb, rocblas_esort_ascending, rocblas_evect_original,
                                                           rocblas_fill_upper, ns, A.as<double>(), ns, bs, 0.0,
                                                           resid.as<double>(), 100, sweeps.as<int>(), lam.as<double>(),
                                                           ns, info.as<int>(), nc);
      rocblas_status t3 = rocblas_dtrsm_strided_batched(rb, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none,
                                                        rocblas_diagonal_non_unit, ns, ns, &one, M.as<double>(), ns, bs,
                                                        A.as<double>(), ns, bs, nc);
      if (t1 != rocblas_status_success || t2 != rocblas_status_success || ev != rocblas_status_success ||
          t3 != rocblas_status_success)
        fail(STMG_E_HIP, "batched reduction or Jacobi eigensolver failed");
      inf = download<int>(info.get(), g.ncells, s);
      for (long long c = 0; c < g.ncells && bad_cell < 0; ++c)
        if (inf[c] != 0) bad_cell = c;
    }
    if (bad_cell >= 0) {       // not positive definite, or not converged: also solved again
      nbad = 1;
      continue;
    }
    for (long long c0 = 0; c0 < g.ncells; c0 += chunk) {
      const int nb = (int)std::min<long long>(chunk, g.ncells - c0);
      const double* Qc = A.as<double>() + c0 * ns * ns;
      rocblas_status g1 = rocblas_dgemm_strided_batched(rb, rocblas_operation_none, rocblas_operation_none, ns, ns, ns,
                                                        &one, M0.as<double>() + c0 * ns * ns, ns, bs, Qc, ns, bs,
                                                        &zero, Tb.as<double>(), ns, bs, nb);
      rocblas_status g2 = rocblas_dgemm_strided_batched(rb, rocblas_operation_transpose, rocblas_operation_none, ns, ns,
                                                        ns, &one, Qc, ns, bs, Tb.as<double>(), ns, bs, &zero,
                                                        Rb.as<double>(), ns, bs, nb);
      rocblas_status g3 = rocblas_dgemm_strided_batched(rb, rocblas_operation_none, rocblas_operation_none, ns, ns, ns,
                                                        &one, A0.as<double>() + c0 * ns * ns, ns, bs, Qc, ns, bs,
                                                        &zero, AQb.as<double>(), ns, bs, nb);
      if (g1 != rocblas_status_success || g2 != rocblas_status_success || g3 != rocblas_status_success)
        fail(STMG_E_HIP, "rocblas_dgemm_strided_batched failed in the eigenpair check");
      asm_eig_check(nb, ns, Rb.as<double>(), AQb.as<double>(), Tb.as<double>(), lam.as<double>() + c0 * ns,
                    EIG_CHECK_TOL, flag.as<int>() + c0, s);
    }
    std::vector<int> fl = download<int>(flag.get(), g.ncells, s);
    nbad = 0;
    for (long long c = 0; c < g.ncells; ++c) nbad += fl[c] != 0;
    if (nbad == 0) break;
  }
  if (bad_cell >= 0)
    fail(STMG_E_ARG, "local smoother block is not positive definite (cell " + std::to_string(bad_cell) + ")");
  if (nbad) fail(STMG_E_HIP, std::to_string(nbad) + " local eigenproblems failed the eigenpair check after 3 solves");
  A0.release();
  M0.release();
  Tb.release();
  Rb.release();
  AQb.release();
  M.release();
  int nt = L.ts->tm.nt_cell;
  DevBuf Mt = upload(L.ts->tm.M_tau.a, s), Nt = upload(L.ts->tm.N_tilde.a, s), bad(sizeof(int));
  STMG_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int), s));
  if (L.has32) {
    L.d32.Q.alloc(sizeof(float) * nblk);
    convert_from_double<float>(A.as<double>(), L.d32.Q.as<float>(), nblk, s);
    L.d32.Tinv.alloc(sizeof(float) * g.ncells * ns * nt * nt);
    asm_tinv<float>(g.ncells, ns, nt, lam.as<double>(), Mt.as<double>(), Nt.as<double>(),
                    L.d32.Tinv.as<float>(), bad.as<int>(), s);
  }
  if (L.has64) {
    L.d64.Tinv.alloc(sizeof(double) * g.ncells * ns * nt * nt);
    asm_tinv<double>(g.ncells, ns, nt, lam.as<double>(), Mt.as<double>(), Nt.as<double>(),
                     L.d64.Tinv.as<double>(), bad.as<int>(), s);
    L.d64.Q = std::move(A);
  }
  std::vector<int> b = download<int>(bad.get(), 1, s);
  if (b[0]) fail(STMG_E_ARG, "singular temporal block in the smoother set-up");
}

template <class T>
void alloc_work(Level& L, int n_t, bool coarsest, bool colour_only) {
  LevelData<T>& d = ldata<T>(L);
  size_t n = (size_t)L.g.nx * n_t * sizeof(T);
  d.u.alloc(n);
  d.r.alloc(n);
  d.f.alloc(n);
  {
    const long long nq = L.g.dim == 3 ? (long long)L.g.n * L.g.n * L.g.n : (long long)L.g.n * L.g.n;
    const size_t bytes = sizeof(T) * L.g.ncells * n_t * nq;
    // the buffer only speeds up the apply: without it (device memory exhausted on a large level,
    // or the colour path requested) the level runs on 2^d colour launches
    if (!colour_only) {
      if (L.g.ncells <= TWO_PHASE_MAX_CELLS) d.cellbuf.alloc(bytes);
      else (void)d.cellbuf.try_alloc(bytes);
    }
  }
  if (!coarsest) {
    d.tmpA.alloc(n);
    d.tmpB.alloc(n);
  }
}

// coarsest level: probe the interior operator column by column, invert on the host
void setup_coarse(stmg_handle* h, Level& L) {
  hipStream_t s = h->stream;
  int n_t = L.n_t();
  std::vector<unsigned char> mask = download<unsigned char>(L.mask.get(), L.g.nx, s);
  std::vector<long long> idx;
  for (int t = 0; t < n_t; ++t)
    for (long long gnode = 0; gnode < L.g.nx; ++gnode)
      if (mask[gnode]) idx.push_back((long long)t * L.g.nx + gnode);
  int m = (int)idx.size();
  if (m > 6000) fail(STMG_E_UNSUPPORTED, "coarsest level too large (" + std::to_string(m) + " unknowns); raise the cell count to a power of two or lower coarse_cells");
  L.cm = m;
  L.cidx = upload(idx, s);
  if (m == 0) return;
  size_t n = (size_t)L.g.nx * n_t;
  DevBuf x(sizeof(double) * n), y(sizeof(double) * n);
  hm::Mat C(m, m);
  fill<double>(x.as<double>(), 0.0, n, s);
  for (int j = 0; j < m; ++j) {
    double one = 1.0, zero = 0.0;
    STMG_HIP(hipMemcpyAsync(x.as<double>() + idx[j], &one, sizeof(double), hipMemcpyHostToDevice, s));
    fill<double>(y.as<double>(), 0.0, n, s);
    st_apply<double>(L.g, L.lt, tdev<double>(L), x.as<double>(), y.as<double>(), 1.0, s);
    std::vector<double> col = download<double>(y.get(), n, s);
    for (int i = 0; i < m; ++i) C(i, j) = col[idx[i]];
    STMG_HIP(hipMemcpyAsync(x.as<double>() + idx[j], &zero, sizeof(double), hipMemcpyHostToDevice, s));
    STMG_HIP(hipStreamSynchronize(s));
  }
  hm::Mat Ci = hm::inverse(C);
  if (L.has64) L.d64.Cinv = upload(Ci.a, s);
  if (L.has32) {
    std::vector<float> f(Ci.a.begin(), Ci.a.end());
    L.d32.Cinv = upload(f, s);
  }
  STMG_HIP(hipStreamSynchronize(s));
}

}  // namespace

void build_hierarchy(stmg_handle* h, const double* vertices, const double* coeff) {
  const stmg_config& cfg = h->cfg;
  hipStream_t s = h->stream;
  int dim = cfg.dim;
  // temporal discretisations: the finest, then (time_mg) k down to its minimum and tau doubled
  // while the number of time cells stays even (Section 3.2, applied below the spatial levels)
  {
    int k = cfg.k, c = cfg.n_time_cells;
    double tau = cfg.tau;
    const int kmin = cfg.time_method == 0 ? 0 : 1;
    for (;;) {
      auto ts = std::make_unique<TSet>();
      ts->tm = hm::temporal(cfg.problem, cfg.time_method, k, c, tau);
      if (ts->tm.n_t > TT_MAX && cfg.time_mg) fail(STMG_E_UNSUPPORTED, "too many temporal DoFs for temporal multigrid");
      make_temporal<double>(ts->tm, ts->tp64, s);
      make_temporal<float>(ts->tm, ts->tp32, s);
      h->tsets.push_back(std::move(ts));
      if (!cfg.time_mg) break;
      if (k > kmin) --k;
      else if (c % 2 == 0) { c /= 2; tau *= 2.0; }
      else break;
    }
    h->tm = h->tsets[0]->tm;
  }
  int fine_cells[3] = {cfg.n_cells[0], cfg.n_cells[1], dim == 3 ? cfg.n_cells[2] : 1};
  long long ncf = (long long)fine_cells[0] * fine_cells[1] * fine_cells[2];
  std::vector<double> coef(ncf, 1.0);
  if (coeff) {
    for (long long c = 0; c < ncf; ++c) {
      if (!(coeff[c] > 0.0) || !std::isfinite(coeff[c])) fail(STMG_E_ARG, "coefficients must be positive and finite");
      coef[c] = coeff[c];
    }
  }
  // level shapes
  struct Shape { int p; int cells[3]; int ratio; int t; };
  std::vector<Shape> shapes;
  Shape cur{cfg.p, {fine_cells[0], fine_cells[1], fine_cells[2]}, 1, 0};
  shapes.push_back(cur);
  while (cur.p > cfg.min_p) {
    cur.p = std::max(cfg.min_p, cur.p / 2);
    shapes.push_back(cur);
  }
  for (;;) {
    bool ok = true;
    for (int d = 0; d < dim; ++d)
      if (cur.cells[d] % 2 != 0 || cur.cells[d] / 2 < cfg.coarse_cells) ok = false;
    if (!ok) break;
    for (int d = 0; d < dim; ++d) cur.cells[d] /= 2;
    cur.ratio *= 2;
    shapes.push_back(cur);
  }
  // temporal levels on the coarsest spatial mesh, if it has an interior node at all
  bool has_interior = true;
  for (int d = 0; d < dim; ++d)
    if ((long long)cur.cells[d] * cur.p + 1 < 3) has_interior = false;
  if (!has_interior) h->tsets.resize(1);
  for (size_t t = 1; t < h->tsets.size(); ++t) {
    cur.t = (int)t;
    shapes.push_back(cur);
  }
  if ((int)shapes.size() > STMG_MAX_LEVELS) fail(STMG_E_UNSUPPORTED, "too many levels");
  std::vector<double> verts_host;
  if (vertices) {
    long long nv = 1;
    for (int d = 0; d < dim; ++d) nv *= fine_cells[d] + 1;
    verts_host.assign(vertices, vertices + nv * dim);
  }
  for (size_t l = 0; l < shapes.size(); ++l) {
    auto L = std::make_unique<Level>();
    L->p = shapes[l].p;
    for (int d = 0; d < 3; ++d) L->cells[d] = shapes[l].cells[d];
    L->ratio = shapes[l].ratio;
    L->ts = h->tsets[shapes[l].t].get();
    init_geom(*L, dim, cfg);
    L->lt = make_level_tables(L->p);
    if (vertices) {
      // even-index subset of the finest vertex lattice
      int r = L->ratio;
      std::vector<double> v;
      int vn[3] = {L->cells[0] + 1, L->cells[1] + 1, dim == 3 ? L->cells[2] + 1 : 1};
      int fn[3] = {fine_cells[0] + 1, fine_cells[1] + 1, dim == 3 ? fine_cells[2] + 1 : 1};
      v.reserve((size_t)vn[0] * vn[1] * vn[2] * dim);
      for (int z = 0; z < vn[2]; ++z)
        for (int y = 0; y < vn[1]; ++y)
          for (int x = 0; x < vn[0]; ++x) {
            size_t src = ((size_t)(z * r) * fn[1] + (size_t)y * r) * fn[0] + (size_t)x * r;
            for (int d = 0; d < dim; ++d) v.push_back(verts_host[src * dim + d]);
          }
      L->verts = upload(v, s);
      L->g.verts = L->verts.as<double>();
    }
    level_coefficients(*L, coef, fine_cells, s);
    L->ct = make_cart_tables(L->lt);
    L->brick = cfg.kernel_path == STMG_PATH_DEFAULT && brick_applicable(L->g);
    if (cfg.asm_variant == 1) {
      // cell mean of the finest coefficient over the ratio^d finest cells of each cell
      const int r = L->ratio;
      L->rho_mean.assign((size_t)L->g.ncells, 0.0);
      for (long long c = 0; c < L->g.ncells; ++c) {
        const int cx = (int)(c % L->cells[0]), cy = (int)((c / L->cells[0]) % L->cells[1]),
                  cz = dim == 3 ? (int)(c / ((long long)L->cells[0] * L->cells[1])) : 0;
        double sum = 0.0;
        int cnt = 0;
        for (int z = 0; z < (dim == 3 ? r : 1); ++z)
          for (int y = 0; y < r; ++y)
            for (int x = 0; x < r; ++x) {
              const long long f = ((long long)(cz * (dim == 3 ? r : 1) + z) * fine_cells[1] + (cy * r + y)) *
                                      fine_cells[0] + (cx * r + x);
              sum += coef[f];
              ++cnt;
            }
        L->rho_mean[c] = sum / cnt;
      }
    }
    if (cfg.asm_variant == 2) {
      // vertex-patch mean of the finest coefficient: the 2 ratio finest cells per axis around
      // each interior vertex
      const int r = L->ratio, rz = dim == 3 ? r : 1;
      const int nv[3] = {L->cells[0] - 1, L->cells[1] - 1, dim == 3 ? L->cells[2] - 1 : 1};
      if (nv[0] >= 1 && nv[1] >= 1 && nv[2] >= 1) {
        L->rho_patch.assign((size_t)nv[0] * nv[1] * nv[2], 0.0);
        for (int vz = 0; vz < nv[2]; ++vz)
          for (int vy = 0; vy < nv[1]; ++vy)
            for (int vx = 0; vx < nv[0]; ++vx) {
              double sum = 0.0;
              int cnt = 0;
              for (int z = 0; z < 2 * rz; ++z)
                for (int y = 0; y < 2 * r; ++y)
                  for (int x = 0; x < 2 * r; ++x) {
                    const long long fz = dim == 3 ? (long long)vz * r + z : 0;
                    const long long f = (fz * fine_cells[1] + ((long long)vy * r + y)) * fine_cells[0] + ((long long)vx * r + x);
                    sum += coef[f];
                    ++cnt;
                  }
              L->rho_patch[((size_t)vz * nv[1] + vy) * nv[0] + vx] = sum / cnt;
            }
      }
    }
    boundary_lists(*L, s);
    L->has64 = h->want64;
    L->has32 = h->want32;
    h->levels.push_back(std::move(L));
  }
  // transfers: level l (fine) <- level l+1 (coarse)
  for (size_t l = 0; l + 1 < h->levels.size(); ++l) {
    Level& F = *h->levels[l];
    Level& C = *h->levels[l + 1];
    if (F.ts != C.ts) {
      F.tkind = 1;
      hm::Mat Pt = hm::temporal_prolongation(F.ts->tm, C.ts->tm);
      F.Pt64 = upload(Pt.a, s);
      std::vector<float> p32(Pt.a.begin(), Pt.a.end());
      F.Pt32 = upload(p32, s);
      continue;
    }
    for (int d = 0; d < dim; ++d) transfer_1d(C.p, C.cells[d], F.p, F.cells[d], F.P[d], F.R[d], s);
    if (dim == 3) {
      build_fused3(F.P, F.PF, s);
      build_fused3(F.R, F.RF, s);
    }
  }
  // smoothers, work vectors, coarse inverse
  for (size_t l = 0; l < h->levels.size(); ++l) {
    Level& L = *h->levels[l];
    bool coarsest = (l + 1 == h->levels.size());
    const bool colour_only = cfg.kernel_path == STMG_PATH_COLOUR;
    if (L.has64) alloc_work<double>(L, L.n_t(), coarsest, colour_only);
    if (L.has32) alloc_work<float>(L, L.n_t(), coarsest, colour_only);
    // the outer FP64 operator of the solver runs on the finest level in every mode
    if (l == 0 && !L.has64 && !L.brick && !colour_only) {
      const long long nq = L.g.dim == 3 ? (long long)L.g.n * L.g.n * L.g.n : (long long)L.g.n * L.g.n;
      const size_t bytes = sizeof(double) * L.g.ncells * L.n_t() * nq;
      if (L.g.ncells <= TWO_PHASE_MAX_CELLS) L.d64.cellbuf.alloc(bytes);
      else (void)L.d64.cellbuf.try_alloc(bytes);
    }
    if (!coarsest) setup_smoother(h, L);
    else setup_coarse(h, L);
  }
  // relaxation
  if (cfg.omega > 0.0) {
    for (auto& L : h->levels) L->omega = cfg.omega;
  } else {
    estimate_omegas(h);
  }
  h->levels.back()->omega = 0.0;
  STMG_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------ level operations

template <class T> void vmult(stmg_handle* h, int level, const T* x, T* y) {
  Level& L = *h->levels[level];
  hipStream_t s = h->stream;
  long long n = L.nst(L.n_t());
  T* cb = ldata<T>(L).cellbuf.template as<T>();
  // the brick and per-cell buffer paths write y themselves
  if (!cb && !L.brick) fill<T>(y, (T)0, n, s);
  if (level == 0) h->ktimer.begin(0, s);
  if (L.brick) st_apply_brick<T>(L.g, L.ct, tdev<T>(L), x, y, (T)1, s, nullptr, true);
  else st_apply<T>(L.g, L.lt, tdev<T>(L), x, y, (T)1, s, cb, nullptr, cb != nullptr);
  if (level == 0) h->ktimer.end(s);
  boundary_axpby<T>(L.bidx.as<int>(), L.nb, L.g.nx, L.n_t(), (T)1, x, (T)0, y, s);
}

// r = f - S u
template <class T> static void residual(stmg_handle* h, Level& L, const T* f, const T* u, T* r) {
  hipStream_t s = h->stream;
  long long n = L.nst(L.n_t());
  T* cb = ldata<T>(L).cellbuf.template as<T>();
  // the brick and per-cell buffer paths read f themselves
  if (!cb && !L.brick) copy<T>(f, r, n, s);
  bool fine = (&L == h->levels[0].get());
  if (fine) h->ktimer.begin(0, s);
  if (L.brick) st_apply_brick<T>(L.g, L.ct, tdev<T>(L), u, r, (T)-1, s, f, true);
  else st_apply<T>(L.g, L.lt, tdev<T>(L), u, r, (T)-1, s, cb, f, cb != nullptr);
  if (fine) h->ktimer.end(s);
  boundary_axpby<T>(L.bidx.as<int>(), L.nb, L.g.nx, L.n_t(), (T)-1, u, (T)1, r, s);
}

// u += omega * ASM(r); u_zero: u is zero on entry (not read on the per-cell buffer path)
template <class T> static void asm_step(stmg_handle* h, Level& L, const T* r, T* u, bool u_zero = false) {
  LevelData<T>& d = ldata<T>(L);
  T* cb = h->cfg.asm_variant == 2 ? nullptr : d.cellbuf.template as<T>();   // patches add into u
  const bool u_zero_in = u_zero;       // the brick smoother writes u itself
  const bool brick_fdm = h->cfg.asm_variant == 1 && h->cfg.kernel_path == STMG_PATH_DEFAULT &&
                         fdm_brick_applicable(L.g, L.ts->tm.nt_cell);
  if (u_zero && !cb && !brick_fdm) fill<T>(u, (T)0, L.nst(L.n_t()), h->stream);
  u_zero = u_zero && cb;
  h->timer.mark(TB_SMOOTH, h->stream);
  bool fine = (&L == h->levels[0].get());
  if (fine) h->ktimer.begin(1, h->stream);
  if (brick_fdm)
    asm_apply_fdm_brick<T>(L.g, L.n_t(), L.ts->tm.nt_cell, L.ts->tm.M_tau.a.data(), L.ts->tm.N_tilde.a.data(),
                           d.fq.template as<T>(), d.fl.template as<T>(), d.frho.template as<T>(), r, u,
                           (T)L.omega, u_zero_in, h->stream);
  else if (h->cfg.asm_variant == 2)
    asm_apply_patch<T>(L.g, L.n_t(), L.ts->tm.nt_cell, d.fq.template as<T>(), d.fl.template as<T>(),
                       d.frho.template as<T>(), d.ftm.template as<T>(), r, u, (T)L.omega, h->stream);
  else if (h->cfg.asm_variant == 1)
    asm_apply_fdm<T>(L.g, L.n_t(), L.ts->tm.nt_cell, d.fq.template as<T>(), d.fl.template as<T>(),
                     d.frho.template as<T>(), d.ftm.template as<T>(), r, u, (T)L.omega, h->stream, cb,
                     u_zero);
  else
    asm_apply<T>(L.g, L.n_t(), L.ts->tm.nt_cell, d.Q.template as<T>(), d.Tinv.template as<T>(), r, u,
                 (T)L.omega, h->stream, cb, u_zero);
  if (fine) h->ktimer.end(h->stream);
  boundary_axpby<T>(L.bidx.as<int>(), L.nb, L.g.nx, L.n_t(), (T)L.omega, r, (T)1, u, h->stream);
  h->timer.mark(TB_GMG, h->stream);
}

template <class T> void smooth(stmg_handle* h, int level, const T* b, T* x, int steps) {
  Level& L = *h->levels[level];
  LevelData<T>& d = ldata<T>(L);
  for (int i = 0; i < steps; ++i) {
    residual<T>(h, L, b, x, d.r.template as<T>());
    asm_step<T>(h, L, d.r.template as<T>(), x);
  }
}

// One iteration of the multigrid method as a stationary solver on the finest level:
// r = b - S x, z = V r, x <- x + z.
template <class T> void mg_step(stmg_handle* h, const T* b, T* x, T* r, T* z) {
  Level& L = *h->levels[0];
  residual<T>(h, L, b, x, r);
  vcycle<T>(h, 0, r, z);
  axpby<T>((T)1, z, (T)1, x, (long long)L.n_t() * L.g.nx, h->stream);
}
template void mg_step<double>(stmg_handle*, const double*, double*, double*, double*);
template void mg_step<float>(stmg_handle*, const float*, float*, float*, float*);

template <class T> std::array<T3Axis, 3> fused_axes(const Fused3& F) {
  std::array<T3Axis, 3> a;
  for (int d = 0; d < 3; ++d)
    a[d] = T3Axis{F.lo[d].as<int>(), F.hi[d].as<int>(), F.col[d].as<int>(),
                  std::is_same<T, double>::value ? F.w64[d].get() : F.w32[d].get()};
  return a;
}

template <class T> void prolongate(stmg_handle* h, int level, const T* coarse, T* fine, bool accumulate) {
  Level& F = *h->levels[level];
  Level& C = *h->levels[level + 1];
  LevelData<T>& d = ldata<T>(F);
  hipStream_t s = h->stream;
  if (F.tkind == 1) {
    const T* P = std::is_same<T, double>::value ? (const T*)F.Pt64.get() : (const T*)F.Pt32.get();
    time_transfer<T>(P, F.n_t(), C.n_t(), F.g.nx, F.mask.as<unsigned char>(), coarse, fine, accumulate ? 1 : 0, s);
    return;
  }
  int n_t = F.n_t();
  int dim = F.g.dim;
  if (dim == 3 && F.PF.pl.ok) {
    tensor3<T>(coarse, fine, n_t, C.g.nn, F.g.nn, F.PF.pl, fused_axes<T>(F.PF).data(), accumulate, s);
    return;
  }
  const T* in = coarse;
  int dims[3] = {C.g.nn[0], C.g.nn[1], C.g.nn[2]};
  T* bufs[2] = {d.tmpA.template as<T>(), d.tmpB.template as<T>()};
  for (int ax = 0; ax < dim; ++ax) {
    bool last = (ax == dim - 1);
    T* out = last ? fine : bufs[ax & 1];
    const Transfer1D& tr = F.P[ax];
    const T* w = std::is_same<T, double>::value ? (const T*)tr.w64.get() : (const T*)tr.w32.get();
    sweep1d<T>(in, out, n_t, dims, ax, tr.len_out, tr.ptr.as<int>(), tr.col.as<int>(), w, tr.nnz, tr.max_row, last && accumulate, s);
    dims[ax] = tr.len_out;
    in = out;
  }
}

template <class T> void restrict_(stmg_handle* h, int level, const T* fine, T* coarse) {
  Level& F = *h->levels[level];
  Level& C = *h->levels[level + 1];
  LevelData<T>& d = ldata<T>(F);
  hipStream_t s = h->stream;
  if (F.tkind == 1) {
    const T* P = std::is_same<T, double>::value ? (const T*)F.Pt64.get() : (const T*)F.Pt32.get();
    time_transfer<T>(P, F.n_t(), C.n_t(), F.g.nx, F.mask.as<unsigned char>(), fine, coarse, 2, s);
    return;
  }
  int n_t = F.n_t();
  int dim = F.g.dim;
  if (dim == 3 && F.RF.pl.ok) {
    tensor3<T>(fine, coarse, n_t, F.g.nn, C.g.nn, F.RF.pl, fused_axes<T>(F.RF).data(), false, s);
    return;
  }
  const T* in = fine;
  int dims[3] = {F.g.nn[0], F.g.nn[1], F.g.nn[2]};
  T* bufs[2] = {d.tmpA.template as<T>(), d.tmpB.template as<T>()};
  for (int ax = 0; ax < dim; ++ax) {
    bool last = (ax == dim - 1);
    T* out = last ? coarse : bufs[ax & 1];
    const Transfer1D& tr = F.R[ax];
    const T* w = std::is_same<T, double>::value ? (const T*)tr.w64.get() : (const T*)tr.w32.get();
    sweep1d<T>(in, out, n_t, dims, ax, tr.len_out, tr.ptr.as<int>(), tr.col.as<int>(), w, tr.nnz, tr.max_row, false, s);
    dims[ax] = tr.len_out;
    in = out;
  }
}

// Alg. stmg on level `level` with zero initial guess: u = V(f)
template <class T> void vcycle(stmg_handle* h, int level, const T* f, T* u) {
  Level& L = *h->levels[level];
  LevelData<T>& d = ldata<T>(L);
  hipStream_t s = h->stream;
  int n_t = L.n_t();
  if (level + 1 == (int)h->levels.size()) {
    coarse_apply<T>(d.Cinv.template as<T>(), L.cidx.as<long long>(), L.cm, f, u, s);
    boundary_axpby<T>(L.bidx.as<int>(), L.nb, L.g.nx, n_t, (T)1, f, (T)0, u, s);
    return;
  }
  const int nu = h->cfg.n_smooth;
  // pre-smoothing from u = 0: the first step needs no residual (and, on the per-cell buffer
  // path, neither a zero fill nor a read of u)
  asm_step<T>(h, L, f, u, true);
  for (int i = 1; i < nu; ++i) {
    residual<T>(h, L, f, u, d.r.template as<T>());
    asm_step<T>(h, L, d.r.template as<T>(), u);
  }
  residual<T>(h, L, f, u, d.r.template as<T>());
  Level& C = *h->levels[level + 1];
  LevelData<T>& dc = ldata<T>(C);
  restrict_<T>(h, level, d.r.template as<T>(), dc.f.template as<T>());
  vcycle<T>(h, level + 1, dc.f.template as<T>(), dc.u.template as<T>());
  prolongate<T>(h, level, dc.u.template as<T>(), u, true);
  for (int i = 0; i < nu; ++i) {
    residual<T>(h, L, f, u, d.r.template as<T>());
    asm_step<T>(h, L, d.r.template as<T>(), u);
  }
}

template void vmult<double>(stmg_handle*, int, const double*, double*);
template void vmult<float>(stmg_handle*, int, const float*, float*);
template void smooth<double>(stmg_handle*, int, const double*, double*, int);
template void smooth<float>(stmg_handle*, int, const float*, float*, int);
template void vcycle<double>(stmg_handle*, int, const double*, double*);
template void vcycle<float>(stmg_handle*, int, const float*, float*);
template void prolongate<double>(stmg_handle*, int, const double*, double*, bool);
template void prolongate<float>(stmg_handle*, int, const float*, float*, bool);
template void restrict_<double>(stmg_handle*, int, const double*, double*);
template void restrict_<float>(stmg_handle*, int, const float*, float*);

// ------------------------------------------------------------------ relaxation estimate

namespace {
// eigenvalues of a small upper Hessenberg matrix by complex shifted QR (Wilkinson shifts)
std::vector<std::complex<double>> hessenberg_eigs(const hm::Mat& H0) {
  int n = H0.r;
  using C = std::complex<double>;
  std::vector<C> H((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) H[(size_t)i * n + j] = H0(i, j);
  auto at = [&](int i, int j) -> C& { return H[(size_t)i * n + j]; };
  std::vector<C> eig;
  int hi = n - 1, iter = 0;
  while (hi >= 0) {
    if (hi == 0) { eig.push_back(at(0, 0)); break; }
    int l = hi;
    while (l > 0) {
      double sc = std::abs(at(l, l)) + std::abs(at(l - 1, l - 1));
      if (std::abs(at(l, l - 1)) <= 1e-15 * (sc > 0 ? sc : 1.0)) { at(l, l - 1) = 0; break; }
      --l;
    }
    if (l == hi || ++iter > 500 * n) { eig.push_back(at(hi, hi)); --hi; iter = 0; continue; }
    C a = at(hi - 1, hi - 1), b = at(hi - 1, hi), c = at(hi, hi - 1), d = at(hi, hi);
    C tr = a + d, det = a * d - b * c;
    C disc = std::sqrt(tr * tr / 4.0 - det);
    C e1 = tr / 2.0 + disc, e2 = tr / 2.0 - disc;
    C mu = (std::abs(e1 - d) < std::abs(e2 - d)) ? e1 : e2;
    // QR step on rows/cols l..hi of H - mu I with Givens rotations, then RQ + mu I
    for (int i = l; i <= hi; ++i) at(i, i) -= mu;
    std::vector<C> cs(hi - l), sn(hi - l);
    for (int k = l; k < hi; ++k) {
      C x = at(k, k), y = at(k + 1, k);
      double r = std::sqrt(std::norm(x) + std::norm(y));
      C cc = r > 0 ? x / r : C(1.0), ss = r > 0 ? y / r : C(0.0);
      cs[k - l] = cc;
      sn[k - l] = ss;
      for (int j = k; j < n; ++j) {
        C t1 = at(k, j), t2 = at(k + 1, j);
        at(k, j) = std::conj(cc) * t1 + std::conj(ss) * t2;
        at(k + 1, j) = -ss * t1 + cc * t2;
      }
    }
    for (int k = l; k < hi; ++k) {
      C cc = cs[k - l], ss = sn[k - l];
      for (int i = 0; i <= std::min(k + 2, hi); ++i) {
        C t1 = at(i, k), t2 = at(i, k + 1);
        at(i, k) = t1 * cc + t2 * ss;
        at(i, k + 1) = -t1 * std::conj(ss) + t2 * std::conj(cc);
      }
    }
    for (int i = l; i <= hi; ++i) at(i, i) += mu;
  }
  return eig;
}
}  // namespace

// omega_l = 2 / (lambda_max + lambda_min) of ASM * S (eq. relaxation), from the real parts of
// the Ritz values of 15 Arnoldi steps with a deterministic start vector, clamped to (0, 1];
// with a negative omega in the configuration, omega_l = |omega| / lambda_max instead (a
// smoothing-oriented choice that damps the top of the spectrum, see the header)
void estimate_omegas(stmg_handle* h) {
  hipStream_t s = h->stream;
  const int steps = 15;
  DevBuf red(sizeof(double) * RED_BLOCKS * PS), dots(sizeof(double) * 64);
  for (size_t l = 0; l + 1 < h->levels.size(); ++l) {
    Level& L = *h->levels[l];
    const int n_t = L.n_t();
    long long n = L.nst(n_t);
    DevBuf V(sizeof(double) * n * (steps + 1)), r(sizeof(double) * n), z(sizeof(double) * n);
    DevBuf r32, z32;
    if (!L.has64) { r32.alloc(sizeof(float) * n); z32.alloc(sizeof(float) * n); }
    // start vector 1 + sin(0.7 g + 1.3 i + 0.1) / 2 on interior DoFs
    std::vector<double> v0(n);
    std::vector<unsigned char> mask = download<unsigned char>(L.mask.get(), L.g.nx, s);
    for (int i = 0; i < n_t; ++i)
      for (long long g = 0; g < L.g.nx; ++g)
        v0[(size_t)i * L.g.nx + g] = mask[g] ? 1.0 + 0.5 * std::sin(0.7 * g + 1.3 * i + 0.1) : 0.0;
    double nrm = 0.0;
    for (double v : v0) nrm += v * v;
    nrm = std::sqrt(nrm);
    for (double& v : v0) v /= nrm;
    double* Vd = V.as<double>();
    STMG_HIP(hipMemcpyAsync(Vd, v0.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
    hm::Mat H(steps + 1, steps);
    double save = L.omega;
    L.omega = 1.0;
    int m = steps;
    for (int j = 0; j < steps; ++j) {
      vmult<double>(h, (int)l, Vd + j * n, r.as<double>());
      if (L.has64) {
        fill<double>(z.as<double>(), 0.0, n, s);
        asm_step<double>(h, L, r.as<double>(), z.as<double>());
      } else {
        cast_d2f(r.as<double>(), r32.as<float>(), n, s);
        fill<float>(z32.as<float>(), 0.0f, n, s);
        asm_step<float>(h, L, r32.as<float>(), z32.as<float>());
        cast_f2d(z32.as<float>(), z.as<double>(), n, s);
      }
      // classical Gram-Schmidt, twice
      std::vector<double> hc(j + 2, 0.0);
      for (int pass = 0; pass < 2; ++pass) {
        multi_dot(Vd, n, j + 1, z.as<double>(), n, dots.as<double>(), red.as<double>(), s);
        std::vector<double> hv = download<double>(dots.get(), j + 1, s);
        multi_axpy_neg(Vd, n, j + 1, dots.as<double>(), z.as<double>(), n, s);
        for (int i = 0; i <= j; ++i) hc[i] += hv[i];
      }
      multi_dot(z.as<double>(), n, 1, z.as<double>(), n, dots.as<double>(), red.as<double>(), s);
      double nz = std::sqrt(download<double>(dots.get(), 1, s)[0]);
      for (int i = 0; i <= j; ++i) H(i, j) = hc[i];
      H(j + 1, j) = nz;
      if (!(nz > 1e-12)) { m = j + 1; break; }
      axpby<double>(1.0 / nz, z.as<double>(), 0.0, Vd + (j + 1) * n, n, s);
    }
    L.omega = save;
    hm::Mat Hm(m, m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) Hm(i, j) = H(i, j);
    auto ev = hessenberg_eigs(Hm);
    double lmax = -1e300, lmin = 1e300;
    for (auto& e : ev) { lmax = std::max(lmax, e.real()); lmin = std::min(lmin, e.real()); }
    // eq. relaxation (omega field == 0); omega field < 0 selects |omega| / lambda_max instead
    double om = h->cfg.omega < 0.0 ? -h->cfg.omega / lmax : 2.0 / (lmax + lmin);
    if (!std::isfinite(om)) om = 1.0;
    L.omega = std::min(1.0, std::max(1e-3, om));
  }
}

}  // namespace stmg
