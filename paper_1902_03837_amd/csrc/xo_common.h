// Internal helpers shared by the xo HIP sources: error state, checked HIP
// calls, per-stream workspace, complex arithmetic on device.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/xo.h"

namespace xo {

// ----------------------------------------------------------------- errors --
void set_error(const char* fmt, ...);
void clear_error();

struct Status {
  int code;
};

#define XO_TRY_HIP(expr)                                                         \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      ::xo::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),     \
                      __FILE__, __LINE__);                                       \
      return XO_ERR_HIP;                                                         \
    }                                                                            \
  } while (0)

#define XO_ARG(cond, ...)                                                        \
  do {                                                                           \
    if (!(cond)) {                                                               \
      ::xo::set_error(__VA_ARGS__);                                              \
      return XO_ERR_ARG;                                                         \
    }                                                                            \
  } while (0)

#define XO_CHECK_LAUNCH()                                                        \
  do {                                                                           \
    hipError_t e_ = hipGetLastError();                                           \
    if (e_ != hipSuccess) {                                                      \
      ::xo::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_),  \
                      __FILE__, __LINE__);                                       \
      return XO_ERR_HIP;                                                         \
    }                                                                            \
  } while (0)

#define XO_RET(expr)                                                             \
  do {                                                                           \
    int r_ = (expr);                                                             \
    if (r_ != XO_OK) return r_;                                                  \
  } while (0)

// -------------------------------------------------------------- workspace --
// Device scratch owned by the library, one growable buffer per (device, stream,
// slot). Growth synchronises the stream before freeing the old buffer, because
// kernels already enqueued on it may still read it.
int workspace(hipStream_t s, int slot, size_t bytes, void** out);
// Pinned host scratch for small flags read back after a synchronisation.
int host_flags(hipStream_t s, size_t bytes, void** out);

// Cached device copy of an immutable host table (geometry, index lists),
// keyed by content. Returned pointer stays valid until xo_release_workspace.
int device_table(const void* host, size_t bytes, hipStream_t s, const void** out);
// 64-bit hash of a byte range (cache keys; equality is always checked in full).
uint64_t content_hash(const void* p, size_t n);
// Counter bumped by xo_release_workspace: pointers from device_table obtained
// under an older value are gone.
unsigned table_generation();

// Event bracket around one kernel launch when timing is enabled (no-op otherwise).
struct KernelTimer {
  KernelTimer(const char* name, hipStream_t s);
  ~KernelTimer();
  const char* name;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
};

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ----------------------------------------------------------- device math --
template <typename T>
struct cplx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
// acc += a * b
template <typename T>
__device__ __forceinline__ void cfma(cplx<T>& acc, cplx<T> a, cplx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <typename T>
__device__ __forceinline__ void cfma_conj(cplx<T>& acc, cplx<T> a, cplx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}

// Loads and stores through the global address space. Pointers that reach a
// kernel inside descriptor tables are otherwise generic (flat) accesses, which
// also count against the LDS wait counter and serialise with LDS reads.
// T must be a scalar or a clang vector type.
template <typename T>
__device__ __forceinline__ T gld(const void* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ void gst(void* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}

__host__ __device__ inline int pmod(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

}  // namespace xo
