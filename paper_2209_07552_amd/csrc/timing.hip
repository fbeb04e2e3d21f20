// Per-kernel timing for profiling: while enabled, the SpMV path brackets each
// kernel it launches (or only the kernel named by msrep_timing_only) with a
// pair of HIP events recorded on the caller's stream; msrep_timing_read
// waits for them and totals the elapsed times by kernel name.  Off by
// default, so the SpMV path records nothing.  Every event record adds a gap
// of a few microseconds between kernels, hence the filter.
//
// msrep_probe_stream: plain 16-byte streams (a read and a copy) that give
// the HBM rate reachable on this GPU, the practical ceiling for the SpMV
// kernels' streams.
#include <atomic>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace msrep {
namespace {

struct Mark {
  const char *name;
  hipEvent_t e0, e1;
};

struct Timing {
  std::mutex mu;
  std::atomic<bool> on{false};
  std::vector<hipEvent_t> pool;  // events free for reuse
  std::vector<Mark> marks;       // recorded, not yet read
  hipEvent_t open = nullptr;     // begin event of the launch in progress
  std::string only;              // the one kernel to time ("" = all)
};

Timing &timing() {
  static Timing t;
  return t;
}

hipEvent_t take_event(Timing &t) {
  if (!t.pool.empty()) {
    hipEvent_t e = t.pool.back();
    t.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

void recycle(Timing &t) {
  for (const Mark &m : t.marks) {
    t.pool.push_back(m.e0);
    t.pool.push_back(m.e1);
  }
  t.marks.clear();
  if (t.open) t.pool.push_back(t.open);
  t.open = nullptr;
}

}  // namespace

void timing_begin(const char *name, hipStream_t s) {
  Timing &t = timing();
  if (!t.on.load(std::memory_order_relaxed)) return;
  std::lock_guard<std::mutex> g(t.mu);
  if (!t.only.empty() && t.only != name) return;
  if (t.open) t.pool.push_back(t.open);
  t.open = nullptr;
  hipEvent_t e = take_event(t);
  if (e && hipEventRecord(e, s) == hipSuccess)
    t.open = e;
  else if (e)
    t.pool.push_back(e);
}

void timing_end(const char *name, hipStream_t s) {
  Timing &t = timing();
  if (!t.on.load(std::memory_order_relaxed)) return;
  std::lock_guard<std::mutex> g(t.mu);
  if (!t.only.empty() && t.only != name) return;
  if (!t.open) return;
  hipEvent_t e = take_event(t);
  if (e && hipEventRecord(e, s) == hipSuccess) {
    t.marks.push_back(Mark{name, t.open, e});
  } else {
    t.pool.push_back(t.open);
    if (e) t.pool.push_back(e);
  }
  t.open = nullptr;
}

}  // namespace msrep

using namespace msrep;

extern "C" msrep_status msrep_timing(int32_t enable) {
  Timing &t = timing();
  std::lock_guard<std::mutex> g(t.mu);
  for (const Mark &m : t.marks) (void)hipEventSynchronize(m.e1);
  recycle(t);
  t.on.store(enable != 0);
  return ok();
}

extern "C" msrep_status msrep_timing_only(const char *kernel) {
  Timing &t = timing();
  std::lock_guard<std::mutex> g(t.mu);
  t.only = kernel ? kernel : "";
  return ok();
}

extern "C" int32_t msrep_timing_read(msrep_kernel_time *out, int32_t cap) {
  if (cap < 0 || (cap > 0 && !out)) return fail(MSREP_ERR_ARG, "msrep_timing_read: bad buffer");
  Timing &t = timing();
  std::lock_guard<std::mutex> g(t.mu);
  std::vector<msrep_kernel_time> agg;
  msrep_status err = MSREP_OK;
  for (const Mark &m : t.marks) {
    float ms = 0.f;
    if (hipEventSynchronize(m.e1) != hipSuccess || hipEventElapsedTime(&ms, m.e0, m.e1) != hipSuccess) {
      err = fail(MSREP_ERR_HIP, "msrep_timing_read: event timing failed");
      break;
    }
    size_t i = 0;
    while (i < agg.size() && std::strncmp(agg[i].name, m.name, sizeof agg[i].name) != 0) ++i;
    if (i == agg.size()) {
      msrep_kernel_time k{};
      std::strncpy(k.name, m.name, sizeof k.name - 1);
      agg.push_back(k);
    }
    agg[i].calls += 1;
    agg[i].total_ms += ms;
  }
  recycle(t);
  if (err) return err;
  for (size_t i = 0; i < agg.size() && static_cast<int32_t>(i) < cap; ++i) out[i] = agg[i];
  ok();
  return static_cast<int32_t>(agg.size());
}

namespace msrep {
namespace {

// One pass over n 16-byte words; the xor of everything read decides a store
// that never happens for real data, so the loads cannot be dropped.
__global__ __launch_bounds__(256) void probe_read(const u32x4 *__restrict__ a, size_t n,
                                                  u32x4 *__restrict__ sink) {
  u32x4 acc = {0u, 0u, 0u, 0u};
  for (size_t i = blockIdx.x * size_t(256) + threadIdx.x; i < n; i += size_t(gridDim.x) * 256) {
    const u32x4 v = __builtin_nontemporal_load(a + i);
    acc.x ^= v.x;
    acc.y ^= v.y;
    acc.z ^= v.z;
    acc.w ^= v.w;
  }
  if ((acc.x & acc.y & acc.z & acc.w) == 0xffffffffu) sink[0] = acc;
}

__global__ __launch_bounds__(256) void probe_copy(const u32x4 *__restrict__ a, size_t n,
                                                  u32x4 *__restrict__ b) {
  for (size_t i = blockIdx.x * size_t(256) + threadIdx.x; i < n; i += size_t(gridDim.x) * 256)
    b[i] = __builtin_nontemporal_load(a + i);
}

}  // namespace
}  // namespace msrep

extern "C" msrep_status msrep_probe_stream(const void *src, void *dst, size_t bytes, int32_t mode,
                                           int32_t blocks, void *stream) {
  if (!src || !dst || (reinterpret_cast<uintptr_t>(src) & 15) ||
      (reinterpret_cast<uintptr_t>(dst) & 15))
    return fail(MSREP_ERR_ARG, "msrep_probe_stream: NULL or misaligned buffer");
  if (bytes == 0 || (bytes & 15) || (mode != 0 && mode != 1) || blocks < 0)
    return fail(MSREP_ERR_ARG, "msrep_probe_stream: bad size, mode or block count");
  if (mode == 1) {
    const char *a = static_cast<const char *>(src);
    const char *b = static_cast<const char *>(dst);
    if (a < b + bytes && b < a + bytes)
      return fail(MSREP_ERR_ARG, "msrep_probe_stream: copy buffers overlap");
  }
  const int g = blocks ? blocks : 65536;
  hipStream_t s = as_stream(stream);
  const size_t n = bytes / 16;
  if (mode == 0)
    hipLaunchKernelGGL(probe_read, dim3(g), dim3(256), 0, s, static_cast<const u32x4 *>(src), n,
                       static_cast<u32x4 *>(dst));
  else
    hipLaunchKernelGGL(probe_copy, dim3(g), dim3(256), 0, s, static_cast<const u32x4 *>(src), n,
                       static_cast<u32x4 *>(dst));
  MSREP_LAUNCHED(mode == 0 ? "probe_read" : "probe_copy");
  return ok();
}
