// Shared internals of libstmg: error plumbing, device buffers, small host helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/stmg.h"

namespace stmg {

// Exceptions never cross the C ABI: every entry point converts them to a status.
struct Error : std::runtime_error {
  stmg_status code;
  Error(stmg_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(stmg_status c, const std::string& m) { throw Error(c, m); }

#define STMG_HIP(expr)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      ::stmg::fail(e_ == hipErrorOutOfMemory ? STMG_E_NOMEM : STMG_E_HIP,                \
                   std::string(#expr) + ": " + hipGetErrorString(e_));                   \
  } while (0)

#define STMG_CHECK_LAUNCH() STMG_HIP(hipGetLastError())

// Owning device allocation (hipMalloc / hipFree).
class DevBuf {
 public:
  DevBuf() = default;
  explicit DevBuf(size_t bytes) { alloc(bytes); }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p_(o.p_), n_(o.n_) { o.p_ = nullptr; o.n_ = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p_ = o.p_; n_ = o.n_; o.p_ = nullptr; o.n_ = 0; }
    return *this;
  }
  void alloc(size_t bytes) {
    release();
    if (bytes == 0) return;
    hipError_t e = hipMalloc(&p_, bytes);
    if (e != hipSuccess) {
      p_ = nullptr;
      fail(STMG_E_NOMEM, "hipMalloc(" + std::to_string(bytes) + " bytes): " + hipGetErrorString(e));
    }
    n_ = bytes;
    total_bytes() += (int64_t)bytes;
  }
  // allocation that may fail without an error: returns false (and clears HIP's last error)
  bool try_alloc(size_t bytes) {
    release();
    if (bytes == 0) return true;
    if (hipMalloc(&p_, bytes) != hipSuccess) {
      p_ = nullptr;
      (void)hipGetLastError();
      return false;
    }
    n_ = bytes;
    total_bytes() += (int64_t)bytes;
    return true;
  }
  void release() {
    if (p_) { (void)hipFree(p_); total_bytes() -= (int64_t)n_; }
    p_ = nullptr;
    n_ = 0;
  }
  template <class T> T* as() const { return static_cast<T*>(p_); }
  void* get() const { return p_; }
  size_t bytes() const { return n_; }
  // library-owned device bytes of the process (handles may be created from several threads)
  static std::atomic<int64_t>& total_bytes() { static std::atomic<int64_t> t{0}; return t; }

 private:
  void* p_ = nullptr;
  size_t n_ = 0;
};

template <class T>
inline DevBuf upload(const std::vector<T>& v, hipStream_t s) {
  DevBuf b(v.size() * sizeof(T));
  if (!v.empty()) {
    STMG_HIP(hipMemcpyAsync(b.get(), v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  }
  return b;
}

template <class T>
inline std::vector<T> download(const void* d, size_t n, hipStream_t s) {
  std::vector<T> v(n);
  if (n) {
    STMG_HIP(hipMemcpyAsync(v.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s));
    STMG_HIP(hipStreamSynchronize(s));
  }
  return v;
}

inline unsigned ceil_div(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace stmg
