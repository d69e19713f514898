// Host-side helpers shared by the C-ABI translation units: the thread-local last error,
// HIP error propagation and a device buffer that grows on demand.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "../../include/kvop.h"

namespace kvop {

inline std::string& last_error() {
  static thread_local std::string e;
  return e;
}

inline kvop_status fail(kvop_status s, const std::string& msg) {
  last_error() = msg;
  return s;
}

#define HIPTRY(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return ::kvop::fail(KVOP_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));  \
  } while (0)

inline int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Device buffer that grows on demand (synchronising the stream before a reallocation).
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  hipError_t reserve(size_t bytes, hipStream_t st) {
    if (bytes <= cap) return hipSuccess;
    if (p) {
      hipError_t e = hipStreamSynchronize(st);
      if (e != hipSuccess) return e;
      (void)hipFree(p);
      p = nullptr;
      cap = 0;
    }
    size_t want = std::max(bytes, cap + cap / 2);
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      e = hipMalloc(&p, bytes);
      if (e != hipSuccess) {
        p = nullptr;
        return e;
      }
      want = bytes;
    }
    cap = want;
    return hipSuccess;
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace kvop
