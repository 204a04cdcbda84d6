// C-ABI plumbing: error state, version, workspace and device-table caches.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "xo_common.h"

namespace xo {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

void clear_error() { g_err[0] = 0; }

static std::mutex g_mu;

struct Buf {
  void* p = nullptr;
  size_t n = 0;
};

static std::map<std::tuple<int, hipStream_t, int>, Buf> g_ws;
static std::map<std::tuple<int, hipStream_t>, Buf> g_hostflags;

struct Table {
  std::vector<unsigned char> host;
  void* dev = nullptr;
};
static std::map<std::tuple<int, uint64_t, size_t>, std::vector<Table>> g_tables;
static unsigned g_table_gen = 0;

unsigned table_generation() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_table_gen;
}

static bool fault_alloc() {
  const char* f = getenv("XO_FAULT");
  return f && strcmp(f, "alloc") == 0;
}

static int dev_alloc(void** p, size_t bytes) {
  if (fault_alloc()) {
    set_error("device allocation of %zu bytes failed (forced by XO_FAULT=alloc)", bytes);
    return XO_ERR_ALLOC;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    *p = nullptr;
    return XO_ERR_ALLOC;
  }
  return XO_OK;
}

int workspace(hipStream_t s, int slot, size_t bytes, void** out) {
  int dev = 0;
  XO_TRY_HIP(hipGetDevice(&dev));
  bytes = align_up(bytes < 256 ? 256 : bytes, 256);
  std::lock_guard<std::mutex> lk(g_mu);
  Buf& b = g_ws[std::make_tuple(dev, s, slot)];
  if (b.n < bytes) {
    if (b.p) {
      XO_TRY_HIP(hipStreamSynchronize(s));
      XO_TRY_HIP(hipFree(b.p));
      b.p = nullptr;
      b.n = 0;
    }
    size_t want = bytes + bytes / 8;  // headroom so small growth does not re-allocate
    XO_RET(dev_alloc(&b.p, want));
    b.n = want;
  }
  *out = b.p;
  return XO_OK;
}

int host_flags(hipStream_t s, size_t bytes, void** out) {
  int dev = 0;
  XO_TRY_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  Buf& b = g_hostflags[std::make_tuple(dev, s)];
  if (b.n < bytes) {
    if (b.p) {
      XO_TRY_HIP(hipStreamSynchronize(s));
      XO_TRY_HIP(hipHostFree(b.p));
      b.p = nullptr;
      b.n = 0;
    }
    XO_TRY_HIP(hipHostMalloc(&b.p, bytes));
    b.n = bytes;
  }
  *out = b.p;
  return XO_OK;
}

// Content hash for the table cache: 64-bit multiply-xorshift over 8-byte words
// (a mismatch only costs a memcmp, equality is always checked in full).
uint64_t content_hash(const void* p, size_t n) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  uint64_t h = 0x9e3779b97f4a7c15ull ^ n;
  size_t i = 0;
  for (; i + 8 <= n; i += 8) {
    uint64_t w;
    memcpy(&w, c + i, 8);
    h ^= w;
    h *= 0xff51afd7ed558ccdull;
    h ^= h >> 32;
  }
  for (; i < n; ++i) {
    h ^= c[i];
    h *= 0xc4ceb9fe1a85ec53ull;
  }
  return h;
}

int device_table(const void* host, size_t bytes, hipStream_t s, const void** out) {
  int dev = 0;
  XO_TRY_HIP(hipGetDevice(&dev));
  uint64_t h = content_hash(host, bytes);
  std::lock_guard<std::mutex> lk(g_mu);
  auto& bucket = g_tables[std::make_tuple(dev, h, bytes)];
  for (auto& t : bucket) {
    if (memcmp(t.host.data(), host, bytes) == 0) {
      *out = t.dev;
      return XO_OK;
    }
  }
  Table t;
  t.host.assign(static_cast<const unsigned char*>(host),
                static_cast<const unsigned char*>(host) + bytes);
  XO_RET(dev_alloc(&t.dev, bytes < 256 ? 256 : bytes));
  hipError_t e = hipMemcpyAsync(t.dev, t.host.data(), bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipFree(t.dev);
    set_error("table upload failed: %s", hipGetErrorString(e));
    return XO_ERR_HIP;
  }
  *out = t.dev;
  bucket.push_back(std::move(t));
  return XO_OK;
}

static bool g_timing = false;
struct TimedEvent {
  std::string name;
  hipEvent_t a, b;
};
static std::vector<TimedEvent> g_events;
static std::vector<hipEvent_t> g_pool;

static hipEvent_t pool_get() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

KernelTimer::KernelTimer(const char* n, hipStream_t st) : name(n), s(st) {
  if (!g_timing) return;
  std::lock_guard<std::mutex> lk(g_mu);
  a = pool_get();
  b = pool_get();
  if (a) (void)hipEventRecord(a, s);
}

KernelTimer::~KernelTimer() {
  if (!a || !b) return;
  (void)hipEventRecord(b, s);
  std::lock_guard<std::mutex> lk(g_mu);
  g_events.push_back({name, a, b});
}

}  // namespace xo

extern "C" {

int xo_timing_enable(int on) {
  xo::g_timing = on != 0;
  return XO_OK;
}

int xo_timing_report(char* buf, int len) {
  std::lock_guard<std::mutex> lk(xo::g_mu);
  std::map<std::string, std::pair<int, double>> acc;
  std::vector<std::string> order;
  for (auto& e : xo::g_events) {
    float ms = 0.f;
    hipError_t r = hipEventSynchronize(e.b);
    if (r == hipSuccess) r = hipEventElapsedTime(&ms, e.a, e.b);
    if (r != hipSuccess) {
      xo::set_error("timing event failed: %s", hipGetErrorString(r));
      return XO_ERR_HIP;
    }
    if (!acc.count(e.name)) order.push_back(e.name);
    acc[e.name].first += 1;
    acc[e.name].second += ms;
    xo::g_pool.push_back(e.a);
    xo::g_pool.push_back(e.b);
  }
  xo::g_events.clear();
  std::string out;
  for (auto& n : order) {
    char line[256];
    snprintf(line, sizeof(line), "%s %d %.6f\n", n.c_str(), acc[n].first, acc[n].second);
    out += line;
  }
  if (buf && len > 0) {
    snprintf(buf, (size_t)len, "%s", out.c_str());
  }
  return XO_OK;
}

const char* xo_last_error(void) { return xo::g_err; }

const char* xo_version(void) { return "xo 0.1.0 (gfx950)"; }

int xo_release_workspace(void) {
  std::lock_guard<std::mutex> lk(xo::g_mu);
  ++xo::g_table_gen;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    xo::set_error("hipDeviceSynchronize failed: %s", hipGetErrorString(e));
    return XO_ERR_HIP;
  }
  for (auto& kv : xo::g_ws)
    if (kv.second.p) (void)hipFree(kv.second.p);
  xo::g_ws.clear();
  for (auto& kv : xo::g_hostflags)
    if (kv.second.p) (void)hipHostFree(kv.second.p);
  xo::g_hostflags.clear();
  for (auto& kv : xo::g_tables)
    for (auto& t : kv.second)
      if (t.dev) (void)hipFree(t.dev);
  xo::g_tables.clear();
  return XO_OK;
}

}  // extern "C"
