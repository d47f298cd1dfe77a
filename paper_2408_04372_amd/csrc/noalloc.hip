// Operator apply for callers that cannot allocate device memory: the per-cell path of the
// operator (every cell's contribution to its own slot, then a node gather in a fixed cell order),
// with the slots in a file-scope static device array instead of memory the library allocates.
// The array's device address is looked up once per device when a handle is created on it; host
// code passes only that address to the kernels.
#include <mutex>
#include <string>

#include "handle.hpp"

namespace stmg {

namespace {

static __device__ __align__(256) unsigned char scratch[STMG_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
void* g_scratch_ptr[MAX_DEVICES] = {};
std::mutex g_scratch_mu;

void* scratch_ptr(int device) {
  if (device < 0 || device >= MAX_DEVICES) fail(STMG_E_UNSUPPORTED, "device index beyond the library's limit");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace

// With `device` current: record the device address of the static scratch array (once per device).
void noalloc_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) fail(STMG_E_UNSUPPORTED, "device index beyond the library's limit");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    fail(STMG_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[device] = p;
}

template <class T> void vmult_noalloc(stmg_handle* h, int level, const T* x, T* y) {
  Level& L = *h->levels[level];
  void* p = scratch_ptr(h->device);
  if (!p) fail(STMG_E_STATE, "the static scratch of this device was not set up (create a handle on it first)");
  const long long nq = L.g.dim == 3 ? (long long)L.g.n * L.g.n * L.g.n : (long long)L.g.n * L.g.n;
  const double need = (double)sizeof(T) * (double)L.g.ncells * L.n_t() * nq;
  if (need > (double)STMG_SCRATCH_BYTES)
    fail(STMG_E_UNSUPPORTED, "level " + std::to_string(level) + " needs " + std::to_string((long long)need) +
                                 " bytes of per-cell scratch; the static scratch holds " +
                                 std::to_string((long long)STMG_SCRATCH_BYTES));
  // every slot of every cell is written before the gather reads it: nothing to clear
  st_apply<T>(L.g, L.lt, tdev<T>(L), x, y, (T)1, h->stream, static_cast<T*>(p), nullptr, true);
  boundary_axpby<T>(L.bidx.as<int>(), L.nb, L.g.nx, L.n_t(), (T)1, x, (T)0, y, h->stream);
}

template void vmult_noalloc<double>(stmg_handle*, int, const double*, double*);
template void vmult_noalloc<float>(stmg_handle*, int, const float*, float*);

}  // namespace stmg
