// msrep_serve: a continuous-batching server for the iterative-solver pattern
// (a request = one pool matrix + `steps` SpMVs against fresh x vectors).
//
//  * Residency: a pool matrix is uploaded into the caller's arena when a
//    request needs it and stays resident (shared by every request on it) until
//    arena space is needed; idle matrices are evicted least recently used.
//  * Admission by bytes: a waiting request is admitted (first come, first
//    served) when its matrix (if not resident), its partitions and its x/y/
//    merge buffers fit in the free arena; one that can never fit fails with
//    MSREP_ERR_BUDGET.  At most max_slots requests are admitted at once.
//  * Continuous batching: every tick runs one step of every ready request in
//    one persistent launch over all their equal-nnz partitions (the batched
//    kernel), so requests that arrive while others run join the next tick.
//    Uploads and partition builds run on a copy stream, overlapping compute.
//  * Each request's arithmetic depends only on its matrix, its partitions and
//    its x: its results are the same alone and in any mix.
// The scheduler is written against an executor interface; the HIP executor
// drives the GPU, and a simulated executor (msrep_serve_simulate) runs the
// same admission and batching logic on a virtual clock, for testing on a CPU.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <type_traits>
#include <vector>

#include "batched.hpp"

namespace msrep {
namespace {

constexpr int kWpb = 4;     // wavefronts per workgroup of the serving kernels
constexpr int kK = 4;       // nonzeros per lane per chunk
constexpr int kRing = 4;    // tick tables in rotation (at most 2 ticks in flight)
constexpr int kInflight = 2;

// ------------------------------------------------------------ x generator
// SplitMix64 output function (Steele, Lea, Flood 2014) applied to a key.
__host__ __device__ inline uint64_t splitmix64(uint64_t key) {
  uint64_t z = key + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ inline double x_value(uint64_t seed, int64_t rid, int32_t step, int64_t c) {
  const uint64_t key = seed ^ (static_cast<uint64_t>(rid) << 40) ^
                       (static_cast<uint64_t>(step) << 24) ^ static_cast<uint64_t>(c);
  const double u = static_cast<double>(splitmix64(key) >> 11) * 0x1.0p-53;
  return 2.0 * u - 1.0;
}

struct FillDesc {
  void *x;
  int64_t rid;
  int32_t n, step;
};

template <typename T>
__global__ void fill_x(const FillDesc *__restrict__ d, uint64_t seed) {
  const FillDesc f = d[blockIdx.y];
  for (int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; c < f.n;
       c += int64_t(gridDim.x) * blockDim.x)
    static_cast<T *>(f.x)[c] = static_cast<T>(x_value(seed, f.rid, f.step, c));
}

// ------------------------------------------------------------------ arena
// First fit over [0, cap) in 256-byte granules; host bookkeeping only.
class Arena {
 public:
  explicit Arena(size_t cap) : cap_(cap) {
    if (cap) free_[0] = cap;
  }
  bool alloc(size_t bytes, size_t *off) {
    bytes = align_up(bytes ? bytes : 1, 256);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t o = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[o + bytes] = rest;
      used_[o] = bytes;
      in_use_ += bytes;
      peak_ = std::max(peak_, in_use_);
      *off = o;
      return true;
    }
    return false;
  }
  void release(size_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t o = off, b = u->second;
    used_.erase(u);
    in_use_ -= b;
    auto nx = free_.lower_bound(o);
    if (nx != free_.end() && o + b == nx->first) {
      b += nx->second;
      free_.erase(nx);
    }
    auto pv = free_.lower_bound(o);
    if (pv != free_.begin()) {
      --pv;
      if (pv->first + pv->second == o) {
        o = pv->first;
        b += pv->second;
        free_.erase(pv);
      }
    }
    free_[o] = b;
  }
  size_t peak() const { return peak_; }
  size_t cap() const { return cap_; }

 private:
  size_t cap_, in_use_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_, used_;
};

// ------------------------------------------------------ scheduler state
enum State { kPending, kWaiting, kLoading, kReady, kDraining, kDone };

struct Resident {  // a pool matrix in the arena
  bool present = false;
  size_t off = 0, bytes = 0;
  int refs = 0;
  int64_t last_use = 0;
  double ready_at = 0;   // simulated executor
  hipEvent_t ev{};       // HIP executor: upload finished
};

struct Req {
  int64_t idx = 0;
  msrep_request r{};
  State st = kPending;
  int32_t np = 1;
  size_t off = 0, bytes = 0;          // x, y, parts, lptr, carry
  size_t x_off, y_off, parts_off, lptr_off, carry_off;
  int32_t enq = 0;                    // steps enqueued
  int64_t last_tick = -1;
  double t_admit = 0, t_done = 0, ready_at = 0;
  hipEvent_t ev{};                    // partitions built
};

size_t mat_bytes(const msrep_mat &A) {
  return align_up(4 * (static_cast<size_t>(A.m) + 1), 256) +
         align_up(4 * static_cast<size_t>(A.nnz), 256) +
         align_up(static_cast<size_t>(value_bytes(A.vtype)) * A.nnz, 256);
}

void layout_req(Req &q, const msrep_mat &A) {
  const size_t xb = vec_bytes(A.vtype);
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o += align_up(b ? b : 1, 256);
    return at;
  };
  q.x_off = take(xb * A.n);
  q.y_off = take(xb * A.m);
  q.parts_off = take(sizeof(msrep_part) * q.np);
  q.lptr_off = take(4 * static_cast<size_t>(msrep_lptr_bound(A.m, q.np)));
  q.carry_off = take(16 * static_cast<size_t>(q.np));
  q.bytes = o;
}

struct Tick {
  int64_t id;
  std::vector<Req *> reqs;
  double end = 0;          // simulated
  hipEvent_t ev{};
};

// ------------------------------------------------------- HIP executor
struct HipExec {
  const msrep_serve_cfg &cfg;
  const msrep_host_mat *pool;
  char *arena;
  hipStream_t copy{}, comp{};
  hipEvent_t t0{};
  std::chrono::steady_clock::time_point w0;
  int32_t vtype;
  // tick tables: device ring (carved from the arena) and pinned staging ring
  size_t table_off = 0, table_bytes = 0;
  char *staging = nullptr;
  int64_t max_items = 0;
  int32_t max_reqs = 0;
  int n_waves_max = 0;

  HipExec(const msrep_serve_cfg &c, const msrep_host_mat *p, int32_t vt)
      : cfg(c), pool(p), arena(static_cast<char *>(c.arena_d)), vtype(vt) {}

  msrep_status init(Arena &A, int64_t items_cap, int32_t reqs_cap) {
    max_items = items_cap;
    max_reqs = reqs_cap;
    MSREP_HIP(hipStreamCreateWithFlags(&copy, hipStreamNonBlocking));
    MSREP_HIP(hipStreamCreateWithFlags(&comp, hipStreamNonBlocking));
    MSREP_HIP(hipEventCreate(&t0));
    table_bytes = slot_bytes();
    if (!A.alloc(table_bytes * kRing, &table_off))
      return fail(MSREP_ERR_BUDGET, "msrep_serve: budget too small for the tick tables");
    MSREP_HIP(hipHostMalloc(reinterpret_cast<void **>(&staging), table_bytes * kRing));
    int dev = 0, per_cu = 0;
    hipDeviceProp_t prop;
    MSREP_HIP(hipGetDevice(&dev));
    MSREP_HIP(hipGetDeviceProperties(&prop, dev));
    const size_t lds = (vtype == MSREP_F64 ? seg_lds_per_wave<MSREP_F64, kK>()
                                           : seg_lds_per_wave<MSREP_F32, kK>()) * kWpb;
    if (vtype == MSREP_F64)
      MSREP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, spmv_batched_persistent<MSREP_F64, kK, true>, kWpb * kWave, lds));
    else
      MSREP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, spmv_batched_persistent<MSREP_F32, kK, true>, kWpb * kWave, lds));
    n_waves_max = std::max(1, per_cu) * kWpb * prop.multiProcessorCount;
    MSREP_HIP(hipEventRecord(t0, comp));
    MSREP_HIP(hipEventSynchronize(t0));
    w0 = std::chrono::steady_clock::now();
    return MSREP_OK;
  }
  size_t slot_bytes() const {
    return align_up(sizeof(BatchMat) * max_reqs, 256) + align_up(sizeof(BatchXY) * max_reqs, 256) +
           align_up(sizeof(FillDesc) * max_reqs, 256) + align_up(sizeof(int2) * max_items, 256) +
           align_up(sizeof(int64_t) * (n_waves_cap() + 1), 256);
  }
  static int n_waves_cap() { return 16384; }
  void shutdown() {
    if (copy) (void)hipStreamSynchronize(copy);
    if (comp) (void)hipStreamSynchronize(comp);
    if (staging) (void)hipHostFree(staging);
    if (t0) (void)hipEventDestroy(t0);
    if (copy) (void)hipStreamDestroy(copy);
    if (comp) (void)hipStreamDestroy(comp);
  }
  double now() const {
    const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - w0).count();
    return s * cfg.time_scale;
  }
  msrep_mat device_mat(int32_t k, const Resident &R) const {
    msrep_mat A = pool[k].A;
    char *b = arena + R.off;
    A.ptr = reinterpret_cast<const int32_t *>(b);
    A.idx = reinterpret_cast<const int32_t *>(b + align_up(4 * (static_cast<size_t>(A.m) + 1), 256));
    A.val = b + align_up(4 * (static_cast<size_t>(A.m) + 1), 256) + align_up(4 * static_cast<size_t>(A.nnz), 256);
    A.idx2 = nullptr;
    return A;
  }
  msrep_status upload(int32_t k, Resident &R) {
    const msrep_mat &H = pool[k].A;
    const msrep_mat D = device_mat(k, R);
    MSREP_HIP(hipMemcpyAsync(const_cast<int32_t *>(D.ptr), H.ptr, 4 * (static_cast<size_t>(H.m) + 1),
                             hipMemcpyHostToDevice, copy));
    if (H.nnz) {
      MSREP_HIP(hipMemcpyAsync(const_cast<int32_t *>(D.idx), H.idx, 4 * static_cast<size_t>(H.nnz),
                               hipMemcpyHostToDevice, copy));
      MSREP_HIP(hipMemcpyAsync(const_cast<void *>(D.val), H.val,
                               static_cast<size_t>(value_bytes(H.vtype)) * H.nnz,
                               hipMemcpyHostToDevice, copy));
    }
    if (!R.ev) MSREP_HIP(hipEventCreateWithFlags(&R.ev, hipEventDisableTiming));
    MSREP_HIP(hipEventRecord(R.ev, copy));
    return MSREP_OK;
  }
  msrep_status prepare(Req &q, const Resident &R) {
    const msrep_mat D = device_mat(q.r.matrix, R);
    char *b = arena + q.off;
    if (msrep_status st = msrep_build_partition(
            &D, q.np, reinterpret_cast<msrep_part *>(b + q.parts_off),
            reinterpret_cast<int32_t *>(b + q.lptr_off), msrep_lptr_bound(D.m, q.np), nullptr, copy))
      return st;
    if (!q.ev) MSREP_HIP(hipEventCreateWithFlags(&q.ev, hipEventDisableTiming));
    MSREP_HIP(hipEventRecord(q.ev, copy));
    return MSREP_OK;
  }
  bool ready(Req &q) { return hipEventQuery(q.ev) == hipSuccess; }

  msrep_status launch(Tick &t, const std::vector<Resident> &res) {
    const int slot = static_cast<int>(t.id % kRing);
    char *hs = staging + slot * table_bytes;
    char *ds = arena + table_off + slot * table_bytes;
    const int32_t cnt = static_cast<int32_t>(t.reqs.size());
    size_t o = 0;
    BatchMat *hm = reinterpret_cast<BatchMat *>(hs + o);
    const size_t om = o;
    o += align_up(sizeof(BatchMat) * max_reqs, 256);
    BatchXY *hxy = reinterpret_cast<BatchXY *>(hs + o);
    const size_t oxy = o;
    o += align_up(sizeof(BatchXY) * max_reqs, 256);
    FillDesc *hf = reinterpret_cast<FillDesc *>(hs + o);
    const size_t of = o;
    o += align_up(sizeof(FillDesc) * max_reqs, 256);
    int2 *hi = reinterpret_cast<int2 *>(hs + o);
    const size_t oi = o;
    o += align_up(sizeof(int2) * max_items, 256);
    int64_t *hw = reinterpret_cast<int64_t *>(hs + o);
    const size_t ow = o;
    std::vector<int64_t> cost;
    int64_t n_items = 0;
    for (int32_t i = 0; i < cnt; ++i) {
      Req &q = *t.reqs[i];
      const msrep_mat D = device_mat(q.r.matrix, res[q.r.matrix]);
      char *b = arena + q.off;
      hm[i] = BatchMat{D.idx, D.val, reinterpret_cast<const msrep_part *>(b + q.parts_off),
                       reinterpret_cast<const int32_t *>(b + q.lptr_off), D.m, D.n, q.np, 0,
                       reinterpret_cast<double *>(b + q.carry_off)};
      hxy[i] = BatchXY{b + q.x_off, b + q.y_off};
      hf[i] = FillDesc{b + q.x_off, q.r.rid, D.n, q.enq};
      for (int32_t p = 0; p < q.np; ++p) {
        hi[n_items++] = int2{i, p};
        cost.push_back(item_cost(D.nnz, D.m, q.np, p));
      }
    }
    const int32_t waves = static_cast<int32_t>(
        std::min<int64_t>({static_cast<int64_t>(n_waves_max), n_waves_cap(), std::max<int64_t>(1, n_items)}));
    equal_work_runs(cost.data(), n_items, waves, hw);
    MSREP_HIP(hipMemcpyAsync(ds, hs, ow + sizeof(int64_t) * (waves + 1), hipMemcpyHostToDevice, comp));
    const BatchMat *dm = reinterpret_cast<const BatchMat *>(ds + om);
    const BatchXY *dxy = reinterpret_cast<const BatchXY *>(ds + oxy);
    const FillDesc *df = reinterpret_cast<const FillDesc *>(ds + of);
    const int2 *di = reinterpret_cast<const int2 *>(ds + oi);
    const int64_t *dw = reinterpret_cast<const int64_t *>(ds + ow);
    const int grid = (waves + kWpb - 1) / kWpb;
    const int gm = static_cast<int>((n_items + 255) / 256);
    if (vtype == MSREP_F64) {
      hipLaunchKernelGGL(fill_x<double>, dim3(16, cnt), dim3(256), 0, comp, df, cfg.seed);
      hipLaunchKernelGGL((spmv_batched_persistent<MSREP_F64, kK, true>), dim3(grid), dim3(kWpb * kWave),
                         (seg_lds_per_wave<MSREP_F64, kK>() * kWpb), comp, dm, dxy, di, dw, waves, 1.0, 0.0);
      hipLaunchKernelGGL((merge_batched<double, true>), dim3(gm), dim3(256), 0, comp, dm, dxy, di,
                         n_items, 1.0, 0.0);
    } else {
      hipLaunchKernelGGL(fill_x<float>, dim3(16, cnt), dim3(256), 0, comp, df, cfg.seed);
      hipLaunchKernelGGL((spmv_batched_persistent<MSREP_F32, kK, true>), dim3(grid), dim3(kWpb * kWave),
                         (seg_lds_per_wave<MSREP_F32, kK>() * kWpb), comp, dm, dxy, di, dw, waves, 1.0, 0.0);
      hipLaunchKernelGGL((merge_batched<float, true>), dim3(gm), dim3(256), 0, comp, dm, dxy, di,
                         n_items, 1.0, 0.0);
    }
    MSREP_LAUNCHED("serve tick");
    if (!t.ev) MSREP_HIP(hipEventCreate(&t.ev));
    MSREP_HIP(hipEventRecord(t.ev, comp));
    return MSREP_OK;
  }
  bool done(Tick &t, double *at) {
    if (hipEventQuery(t.ev) != hipSuccess) return false;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, t0, t.ev);
    *at = ms * 1e-3 * cfg.time_scale;
    return true;
  }
  void release_tick(Tick &t) {
    if (t.ev) (void)hipEventDestroy(t.ev);
    t.ev = nullptr;
  }
  msrep_status keep_y(Req &q, msrep_result &res) {
    if (!cfg.keep_y || !res.y_host) return MSREP_OK;
    const msrep_mat &H = pool[q.r.matrix].A;
    MSREP_HIP(hipMemcpy(res.y_host, arena + q.off + q.y_off, vec_bytes(vtype) * static_cast<size_t>(H.m),
                        hipMemcpyDeviceToHost));
    return MSREP_OK;
  }
  void idle(double until, bool busy) {
    const double wait = until - now();
    if (busy || wait <= 0) {
      std::this_thread::yield();
      return;
    }
    const double s = std::min(wait / cfg.time_scale, 2e-4);
    std::this_thread::sleep_for(std::chrono::duration<double>(s));
  }
  void free_events(std::vector<Resident> &res, std::vector<Req> &reqs) {
    for (auto &r : res)
      if (r.ev) (void)hipEventDestroy(r.ev);
    for (auto &q : reqs)
      if (q.ev) (void)hipEventDestroy(q.ev);
  }
};

// --------------------------------------------------- simulated executor
// Virtual clock: an upload takes bytes / upload_bw, a tick takes a fixed
// launch cost plus 2*nnz / flop_rate per step of each request in it, ticks
// run one after another.
struct SimExec {
  const msrep_host_mat *pool;
  double clock = 0, dev_free = 0, copy_free = 0;
  double upload_bw = 25e9, flop_rate = 5e11, tick_cost = 2e-5;
  int32_t vtype;
  SimExec(const msrep_host_mat *p, int32_t vt) : pool(p), vtype(vt) {}
  msrep_status init(Arena &, int64_t, int32_t) { return MSREP_OK; }
  void shutdown() {}
  double now() const { return clock; }
  msrep_status upload(int32_t k, Resident &R) {
    copy_free = std::max(copy_free, clock) + static_cast<double>(mat_bytes(pool[k].A)) / upload_bw;
    R.ready_at = copy_free;
    return MSREP_OK;
  }
  msrep_status prepare(Req &q, const Resident &R) {
    copy_free = std::max({copy_free, clock, R.ready_at}) + 5e-6;
    q.ready_at = copy_free;
    return MSREP_OK;
  }
  bool ready(Req &q) { return clock >= q.ready_at; }
  msrep_status launch(Tick &t, const std::vector<Resident> &) {
    double work = tick_cost;
    for (Req *q : t.reqs) work += 2.0 * static_cast<double>(pool[q->r.matrix].A.nnz) / flop_rate;
    dev_free = std::max(dev_free, clock) + work;
    t.end = dev_free;
    return MSREP_OK;
  }
  bool done(Tick &t, double *at) {
    if (clock < t.end) return false;
    *at = t.end;
    return true;
  }
  void release_tick(Tick &) {}
  msrep_status keep_y(Req &, msrep_result &) { return MSREP_OK; }
  // advance the virtual clock to the next thing that can happen
  double next_event = 0;
  void idle(double until, bool) { clock = std::max(clock, std::min(until, next_event)); }
  void free_events(std::vector<Resident> &, std::vector<Req> &) {}
};

// ------------------------------------------------------------ scheduler
size_t ex_table_bytes(const HipExec &e) { return e.table_bytes * kRing; }
size_t ex_table_bytes(const SimExec &) { return 0; }

template <class Exec>
msrep_status run_server(Exec &ex, const msrep_serve_cfg &cfg, const msrep_host_mat *pool,
                        int32_t pool_size, const msrep_request *trace, int64_t n_req,
                        msrep_result *results, msrep_serve_stats *stats) {
  Arena arena(cfg.budget_bytes);
  std::vector<Resident> res(pool_size);
  std::vector<Req> reqs(n_req);
  int64_t max_np = 1;
  for (int32_t k = 0; k < pool_size; ++k) {
    const int64_t npw = pool[k].np > 0 ? 0 : std::max(1, cfg.nnz_per_wave);
    const int64_t np = pool[k].np > 0 ? pool[k].np : std::max<int64_t>(1, (pool[k].A.nnz + npw - 1) / npw);
    max_np = std::max(max_np, np);
  }
  const int32_t slots = cfg.max_slots;
  if (msrep_status st = ex.init(arena, max_np * slots, slots)) return st;
  for (int64_t i = 0; i < n_req; ++i) {
    Req &q = reqs[i];
    q.idx = i;
    q.r = trace[i];
    const msrep_host_mat &H = pool[q.r.matrix];
    const int64_t npw = std::max(1, cfg.nnz_per_wave);
    q.np = H.np > 0 ? H.np : static_cast<int32_t>(std::max<int64_t>(1, (H.A.nnz + npw - 1) / npw));
    layout_req(q, H.A);
  }
  std::vector<int64_t> order(n_req);
  for (int64_t i = 0; i < n_req; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return trace[a].t_arrive < trace[b].t_arrive; });
  std::deque<Req *> waiting;
  std::vector<Req *> admitted;  // loading, ready or draining
  std::deque<Tick> inflight;
  int64_t next_arrival = 0, n_finished = 0, tick_id = 0, use_clock = 0;
  int64_t ticks = 0;
  int32_t peak_active = 0;
  msrep_status err = MSREP_OK;

  auto finish = [&](Req &q, msrep_status st, double t) {
    q.st = kDone;
    q.t_done = t;
    results[q.idx].t_arrive = q.r.t_arrive;
    results[q.idx].t_admit = q.t_admit;
    results[q.idx].t_done = t;
    results[q.idx].status = st;
    ++n_finished;
  };
  while (n_finished < n_req && err == MSREP_OK) {
    const double now = ex.now();
    bool progressed = false;
    // arrivals
    while (next_arrival < n_req && trace[order[next_arrival]].t_arrive <= now) {
      Req &q = reqs[order[next_arrival++]];
      q.st = kWaiting;
      waiting.push_back(&q);
      progressed = true;
    }
    // admission, first come first served
    while (!waiting.empty() && static_cast<int32_t>(admitted.size()) < slots) {
      Req &q = *waiting.front();
      Resident &R = res[q.r.matrix];
      const size_t mb = mat_bytes(pool[q.r.matrix].A);
      const size_t need = q.bytes + (R.present ? 0 : mb) + 512;
      const size_t table = arena.cap() >= ex_table_bytes(ex) ? ex_table_bytes(ex) : arena.cap();
      if (q.bytes + mb + 512 > arena.cap() - table) {  // can never fit
        waiting.pop_front();
        finish(q, MSREP_ERR_BUDGET, now);
        progressed = true;
        continue;
      }
      (void)need;
      // make room: evict idle resident matrices, least recently used first
      bool got = false;
      for (;;) {
        size_t mo = 0, ro = 0;
        const bool need_mat = !R.present;
        bool ok_mat = true;
        if (need_mat) ok_mat = arena.alloc(mb, &mo);
        bool ok_req = ok_mat && arena.alloc(q.bytes, &ro);
        if (ok_mat && ok_req) {
          if (need_mat) {
            R.present = true;
            R.off = mo;
            R.bytes = mb;
            if (msrep_status st = ex.upload(q.r.matrix, R)) {
              err = st;
              break;
            }
          }
          q.off = ro;
          got = true;
          break;
        }
        if (ok_mat && need_mat) arena.release(mo);
        int32_t victim = -1;
        for (int32_t k = 0; k < pool_size; ++k)
          if (res[k].present && res[k].refs == 0 && k != q.r.matrix &&
              (victim < 0 || res[k].last_use < res[victim].last_use))
            victim = k;
        if (victim < 0) break;
        arena.release(res[victim].off);
        res[victim].present = false;
      }
      if (err) break;
      if (!got) break;  // wait for running requests to free memory
      R.refs++;
      R.last_use = ++use_clock;
      if (msrep_status st = ex.prepare(q, R)) {
        err = st;
        break;
      }
      q.st = kLoading;
      q.t_admit = now;
      waiting.pop_front();
      admitted.push_back(&q);
      progressed = true;
    }
    if (err) break;
    for (Req *q : admitted)
      if (q->st == kLoading && ex.ready(*q)) {
        q->st = kReady;
        progressed = true;
      }
    // completed ticks, oldest first
    while (!inflight.empty()) {
      double at = 0;
      if (!ex.done(inflight.front(), &at)) break;
      Tick &t = inflight.front();
      for (Req *q : t.reqs) {
        if (q->last_tick == t.id && q->enq == q->r.steps) {
          if (msrep_status st = ex.keep_y(*q, results[q->idx])) err = st;
          finish(*q, MSREP_OK, at);
          res[q->r.matrix].refs--;
          res[q->r.matrix].last_use = ++use_clock;
          arena.release(q->off);
        }
      }
      ex.release_tick(t);
      inflight.pop_front();
      admitted.erase(std::remove_if(admitted.begin(), admitted.end(),
                                    [](Req *q) { return q->st == kDone; }),
                     admitted.end());
      progressed = true;
    }
    // one step of every ready request
    if (static_cast<int>(inflight.size()) < kInflight) {
      Tick t;
      t.id = tick_id;
      for (Req *q : admitted)
        if (q->st == kReady && q->enq < q->r.steps) t.reqs.push_back(q);
      if (!t.reqs.empty()) {
        peak_active = std::max(peak_active, static_cast<int32_t>(t.reqs.size()));
        if (msrep_status st = ex.launch(t, res)) {
          err = st;
          break;
        }
        for (Req *q : t.reqs) {
          q->enq++;
          q->last_tick = t.id;
          if (q->enq == q->r.steps) q->st = kDraining;
        }
        inflight.push_back(std::move(t));
        ++tick_id;
        ++ticks;
        progressed = true;
      }
    }
    if (!progressed) {
      const double until = next_arrival < n_req ? trace[order[next_arrival]].t_arrive : now + 1.0;
      if constexpr (std::is_same_v<Exec, SimExec>) {
        double nx = until;
        for (const Tick &t : inflight) nx = std::min(nx, t.end);
        for (Req *q : admitted)
          if (q->st == kLoading) nx = std::min(nx, q->ready_at);
        ex.next_event = nx;
      }
      ex.idle(until, !inflight.empty());
    }
  }
  ex.shutdown();
  ex.free_events(res, reqs);
  if (err) return err;
  // statistics
  std::vector<double> lat;
  double first = 1e300, last = 0, flops = 0;
  int64_t steps = 0, failed = 0;
  for (int64_t i = 0; i < n_req; ++i) {
    first = std::min(first, trace[i].t_arrive);
    if (results[i].status != MSREP_OK) {
      ++failed;
      continue;
    }
    lat.push_back((results[i].t_done - results[i].t_arrive) * 1e3);
    last = std::max(last, results[i].t_done);
    steps += trace[i].steps;
    flops += 2.0 * static_cast<double>(pool[trace[i].matrix].A.nnz) * trace[i].steps;
  }
  if (stats) {
    std::memset(stats, 0, sizeof *stats);
    std::sort(lat.begin(), lat.end());
    auto pct = [&](double p) {
      if (lat.empty()) return 0.0;
      const size_t i = static_cast<size_t>(std::ceil(p * lat.size())) - 1;
      return lat[std::min(i, lat.size() - 1)];
    };
    const double span = lat.empty() ? 0.0 : std::max(last - first, 1e-12);
    stats->p50_ms = pct(0.50);
    stats->p99_ms = pct(0.99);
    stats->max_ms = lat.empty() ? 0.0 : lat.back();
    double sum = 0;
    for (double v : lat) sum += v;
    stats->mean_ms = lat.empty() ? 0.0 : sum / lat.size();
    stats->makespan_s = span;
    stats->req_per_s = span > 0 ? lat.size() / span : 0.0;
    stats->spmv_per_s = span > 0 ? steps / span : 0.0;
    stats->gflops = span > 0 ? flops / span / 1e9 : 0.0;
    stats->n_done = static_cast<int64_t>(lat.size());
    stats->n_failed = failed;
    stats->ticks = ticks;
    stats->peak_bytes = static_cast<int64_t>(arena.peak());
    stats->peak_active = peak_active;
  }
  return ok();
}

msrep_status check_serve_args(const msrep_serve_cfg *cfg, const msrep_host_mat *pool,
                              int32_t pool_size, const msrep_request *trace, int64_t n_req,
                              msrep_result *results, bool need_arena) {
  if (!cfg || !pool || pool_size <= 0 || (n_req > 0 && (!trace || !results)) || n_req < 0)
    return fail(MSREP_ERR_ARG, "msrep_serve: missing configuration, pool, trace or results");
  if (need_arena && !cfg->arena_d) return fail(MSREP_ERR_ARG, "msrep_serve: arena_d is NULL");
  if (cfg->max_slots < 1 || cfg->max_slots > 4096)
    return fail(MSREP_ERR_ARG, "msrep_serve: max_slots must be 1..4096");
  if (!(cfg->time_scale > 0)) return fail(MSREP_ERR_ARG, "msrep_serve: time_scale must be > 0");
  const int32_t vt = pool[0].A.vtype;
  if (vt != MSREP_F64 && vt != MSREP_F32)
    return fail(MSREP_ERR_UNSUPPORTED, "msrep_serve: pool matrices must be F64 or F32");
  for (int32_t k = 0; k < pool_size; ++k) {
    const msrep_mat &A = pool[k].A;
    if (A.fmt != MSREP_CSR || A.vtype != vt)
      return fail(MSREP_ERR_ARG, "msrep_serve: pool matrix %d must be CSR of the pool's value type", k);
    if (A.m < 0 || A.n < 0 || A.nnz < 0 || A.nnz >= (int64_t(1) << 31) || A.n >= (1 << 24))
      return fail(MSREP_ERR_ARG, "msrep_serve: pool matrix %d has an unsupported shape", k);
    if (need_arena && (!A.ptr || (A.nnz > 0 && (!A.idx || !A.val))))
      return fail(MSREP_ERR_ARG, "msrep_serve: pool matrix %d has NULL arrays", k);
  }
  for (int64_t i = 0; i < n_req; ++i) {
    const msrep_request &r = trace[i];
    if (r.matrix < 0 || r.matrix >= pool_size || r.steps < 1 || r.steps > 65535 || r.rid < 0 ||
        r.rid >= (int64_t(1) << 24))
      return fail(MSREP_ERR_ARG, "msrep_serve: request %lld is malformed", static_cast<long long>(i));
  }
  return MSREP_OK;
}

}  // namespace
}  // namespace msrep

using namespace msrep;

extern "C" msrep_status msrep_serve(const msrep_serve_cfg *cfg, const msrep_host_mat *pool,
                                    int32_t pool_size, const msrep_request *trace, int64_t n_req,
                                    msrep_result *results, msrep_serve_stats *stats) {
  if (msrep_status st = check_serve_args(cfg, pool, pool_size, trace, n_req, results, true)) return st;
  HipExec ex(*cfg, pool, pool[0].A.vtype);
  return run_server(ex, *cfg, pool, pool_size, trace, n_req, results, stats);
}

extern "C" msrep_status msrep_serve_simulate(const msrep_serve_cfg *cfg,
                                             const msrep_host_mat *pool, int32_t pool_size,
                                             const msrep_request *trace, int64_t n_req,
                                             msrep_result *results, msrep_serve_stats *stats,
                                             double upload_bytes_per_s, double flops_per_s,
                                             double tick_seconds) {
  if (msrep_status st = check_serve_args(cfg, pool, pool_size, trace, n_req, results, false)) return st;
  SimExec ex(pool, pool[0].A.vtype);
  if (upload_bytes_per_s > 0) ex.upload_bw = upload_bytes_per_s;
  if (flops_per_s > 0) ex.flop_rate = flops_per_s;
  if (tick_seconds >= 0) ex.tick_cost = tick_seconds;
  return run_server(ex, *cfg, pool, pool_size, trace, n_req, results, stats);
}

extern "C" double msrep_serve_x_value(uint64_t seed, int64_t rid, int32_t step, int64_t c) {
  return x_value(seed, rid, step, c);
}

namespace msrep {
namespace {
template <typename T>
__global__ void fill_x_one(T *__restrict__ x, int32_t n, uint64_t seed, int64_t rid, int32_t step) {
  for (int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; c < n;
       c += int64_t(gridDim.x) * blockDim.x)
    x[c] = static_cast<T>(x_value(seed, rid, step, c));
}
}  // namespace
}  // namespace msrep

extern "C" msrep_status msrep_serve_fill_x(uint64_t seed, int64_t rid, int32_t step, void *x_d,
                                           int32_t n, int32_t vtype, void *stream) {
  if (n < 0 || (n > 0 && !x_d) || (vtype != MSREP_F64 && vtype != MSREP_F32))
    return fail(MSREP_ERR_ARG, "msrep_serve_fill_x: bad vector, size or value type");
  if (n == 0) return ok();
  const int grid = static_cast<int>(std::min<int64_t>((n + 255) / 256, 1024));
  if (vtype == MSREP_F64)
    hipLaunchKernelGGL(fill_x_one<double>, dim3(grid), dim3(256), 0, as_stream(stream),
                       static_cast<double *>(x_d), n, seed, rid, step);
  else
    hipLaunchKernelGGL(fill_x_one<float>, dim3(grid), dim3(256), 0, as_stream(stream),
                       static_cast<float *>(x_d), n, seed, rid, step);
  MSREP_LAUNCHED("fill_x_one");
  return ok();
}
