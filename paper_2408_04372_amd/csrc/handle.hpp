// The library handle: level hierarchy (Section 3, Alg. mg-sequence with spatial and temporal
// levels), per-precision V-cycle data, and the FP64 FGMRES workspace.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <memory>
#include <utility>
#include <vector>

#include "common.hpp"
#include "hostmath.hpp"
#include "kernels.hpp"

namespace stmg {

struct Transfer1D {           // one direction of P (coarse -> fine) or R = P^T (fine -> coarse)
  int len_out = 0, nnz = 0, max_row = 0;   // rows, entries, most entries in one row
  DevBuf ptr, col, w64, w32;
  std::vector<int> ptr_h, col_h;          // host copies (tables of the fused transfer)
  std::vector<double> w_h;
};

struct Fused3 {               // tables of the fused 3D transfer (see Tensor3Plan)
  Tensor3Plan pl;
  DevBuf lo[3], hi[3], col[3], w64[3], w32[3];
};

template <class T>
struct LevelData {            // precision-dependent data of one level
  DevBuf Q, Tinv;             // smoother factors (not on the coarsest level)
  DevBuf u, r, f, tmpA, tmpB; // V-cycle work vectors
  DevBuf Cinv;                // coarsest level only: dense inverse on interior DoFs
  DevBuf cellbuf;             // per-cell contributions (levels with few cells, see st_apply)
  DevBuf fq, fl, frho, ftm;   // separable smoother: 1D eigenvectors / eigenvalues per axis and
                              // boundary case, cell-mean coefficient, temporal blocks M_tau, N~
};

template <class T>
struct TemporalBufs {
  DevBuf mptr, mcol, mval, nptr, ncol, nval;
  DevBuf uptr, ucol, umval, unval;
  TemporalDev<T> dev;
};

// temporal discretisation of a level (the finest one, or a k- / tau-coarsened one)
struct TSet {
  hm::Temporal tm;
  TemporalBufs<double> tp64;
  TemporalBufs<float> tp32;
};

struct Level {
  int p = 1;
  int cells[3] = {1, 1, 1};
  int ratio = 1;              // finest cells per cell of this level, per direction
  GeomDesc g;
  LevelTables lt;
  CartTables ct;              // separable cell matrices (brick operator)
  bool brick = false;         // the operator runs on the brick kernel (3D Cartesian, rho per cell)
  DevBuf verts, rho, bidx, mask;
  long long nb = 0;           // boundary nodes per temporal plane
  long long n_int = 0;        // interior nodes per temporal plane
  double omega = 1.0;
  // transfer between this level (fine) and level+1 (coarse)
  std::array<Transfer1D, 3> P, R;
  Fused3 PF, RF;              // fused 3D transfers (tiles and padded tables)
  // coarsest level
  DevBuf cidx;                // interior DoF indices (full-lattice space-time index)
  int cm = 0;
  LevelData<double> d64;
  LevelData<float> d32;
  bool has64 = false, has32 = false;
  std::vector<double> rho_mean;   // cell mean of the finest coefficient (separable smoother)
  std::vector<double> rho_patch;  // vertex-patch mean of the finest coefficient (patch smoother)
  const TSet* ts = nullptr;       // temporal discretisation of this level
  int tkind = 0;                  // transfer to the next coarser level: 0 in space, 1 in time
  DevBuf Pt64, Pt32;              // temporal prolongation (n_t of this level x n_t of the next)
  int n_t() const { return ts->tm.n_t; }
  long long nst(int n_t) const { return g.nx * n_t; }
};


struct Timer {               // event-based bucket timer for stmg_solve
  std::vector<hipEvent_t> ev;
  std::vector<int> tag;
  size_t used = 0;
  bool on = false;
  void mark(int t, hipStream_t s);
  void reset() { used = 0; }
  void accumulate(double out[4]);
  ~Timer();
};
enum { TB_SMOOTH = 0, TB_GMG = 1, TB_OP = 2, TB_OTHER = 3 };

// event pairs around individual finest-level kernel launches (operator / smoother)
struct KernelTimer {
  std::vector<hipEvent_t> ev;   // 2 per record
  std::vector<int> kind;
  size_t used = 0;
  bool on = false;
  int64_t n[2] = {0, 0};
  double t[2] = {0.0, 0.0};
  void begin(int k, hipStream_t s);
  void end(hipStream_t s);
  void flush();                 // synchronises on the last event and accumulates
  ~KernelTimer();
};

struct CnnState;              // learned stage (cnn.hip)
void cnn_free(CnnState* c);

}  // namespace stmg

struct stmg_handle {
  stmg_config cfg;
  hipStream_t stream = nullptr;
  int device = 0;
  stmg::hm::Temporal tm;                              // finest temporal discretisation
  std::vector<std::unique_ptr<stmg::TSet>> tsets;     // [0]: finest, then the coarser ones
  std::vector<std::unique_ptr<stmg::Level>> levels;
  bool want64 = true, want32 = false;
  // FGMRES workspace (finest level)
  stmg::DevBuf V, Z64, Z32, w, tmp32a, tmp32b, dots, red, hbuf;
  int krylov_m = 0;
  stmg::Timer timer;
  stmg::KernelTimer ktimer;
  double setup_seconds = 0.0;
  int64_t bytes_at_create = 0;
  int eig_resolves = 0;       // batched eigen-solves repeated after a failed eigenpair check
  stmg::CnnState* cnn = nullptr;
  stmg::DevBuf vel;            // wave velocity recovery: M_T^{-1} A_T and the u0 / v0 weights
  stmg::DevBuf rhsc, rhs3x, rhs3y, rhs_mp, rhs_mc, rhs_mv, rhs_np, rhs_nc, rhs_nv;   // slab right-hand sides
  int rhs_mnnz = 0, rhs_nnnz = 0;
  ~stmg_handle();
};

namespace stmg {
// set-up and V-cycle entry points used by the C ABI (hierarchy.hip)
void build_hierarchy(stmg_handle* h, const double* vertices, const double* coeff);
template <class T> void vmult(stmg_handle* h, int level, const T* x, T* y);
// operator apply through the static per-device scratch (noalloc.hip)
void noalloc_init(int device);
template <class T> void vmult_noalloc(stmg_handle* h, int level, const T* x, T* y);
template <class T> void smooth(stmg_handle* h, int level, const T* b, T* x, int steps);
template <class T> void vcycle(stmg_handle* h, int level, const T* f, T* u);
template <class T> void mg_step(stmg_handle* h, const T* b, T* x, T* r, T* z);
template <class T> void prolongate(stmg_handle* h, int level, const T* coarse, T* fine, bool accumulate);
template <class T> void restrict_(stmg_handle* h, int level, const T* fine, T* coarse);
void estimate_omegas(stmg_handle* h);
stmg_status fgmres(stmg_handle* h, const double* b, double* x, stmg_solve_info* info);
void wave_velocity(stmg_handle* h, const double* U, const double* u0, const double* v0, double* V);
void slab_rhs(stmg_handle* h, const double* F, const double* F0, const double* u0, const double* v0, double* b);
void node_coordinates(stmg_handle* h, double* xyz);
void point_values(stmg_handle* h, const double* U, int n_planes, int npts, const double* pts, double* out);
// CSR of the nonzeros of a dense matrix (hierarchy.hip)
template <class T> int upload_csr(const hm::Mat& A, DevBuf& ptr, DevBuf& col, DevBuf& val, hipStream_t s);
// Rows of the 1D prolongation from a coarse (pc, ncc cells) to a fine (pf, ncf cells) lattice along
// one axis, interior nodes only (first and last rows and columns dropped): rows[g] lists
// (coarse node, weight) in increasing coarse node order.  Host only.
std::vector<std::vector<std::pair<int, double>>> transfer_1d_rows(int pc, int ncc, int pf, int ncf);
// learned stage (cnn.hip)
void cnn_create(stmg_handle* h, int n_layers, const int* channels);
long long cnn_param_count(stmg_handle* h);
void cnn_set_params(stmg_handle* h, const float* host, long long n);
void cnn_get_params(stmg_handle* h, float* host, long long n);
double cnn_forward(stmg_handle* h, const double* r, double* z);
void cnn_param_grad(stmg_handle* h, const double* r, const double* dz, float* host);
double cnn_train_step(stmg_handle* h, const double* r, const double* e, double lr);
template <class T> LevelData<T>& ldata(Level& L);
template <class T> const TemporalDev<T>& tdev(const Level& L);
}  // namespace stmg
