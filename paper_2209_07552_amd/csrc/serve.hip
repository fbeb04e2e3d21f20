// msrep_serve and the incremental server (msrep_server_*): continuous
// batching for the iterative-solver pattern (a request = one pool matrix +
// `steps` SpMVs against fresh x vectors).
//
//  * Residency: a pool matrix is uploaded into the caller's arena when a
//    request needs it and stays resident (shared by every request on it) until
//    arena space is needed; idle matrices are evicted least recently used.
//  * Admission by bytes: a waiting request is admitted (first come, first
//    served) when its matrix (if not resident), its partitions and its x/y/
//    merge buffers fit in the free arena; one that can never fit fails with
//    MSREP_ERR_BUDGET.  At most max_slots requests are admitted at once.
//  * Continuous batching: every tick runs the next steps of every ready
//    request in one persistent launch over all their equal-nnz partitions,
//    so requests that arrive while others run join the next tick.  A
//    request's steps are independent SpMVs: those of one tick are the
//    columns of a multi-vector product, run as passes of up to 8 columns
//    side by side, so its matrix is read once per 8 steps, not once per
//    step.  How many steps of each request a tick runs follows the load: as
//    many as steps_per_tick allows while the tick's items fit the resident
//    wavefronts, else 8.  A request's device descriptor is written once, when
//    it is admitted; a tick passes only its entries (slot, first step,
//    steps), in the kernel arguments, so a tick costs three launches and one
//    event record.
//    Uploads and partition builds run on a copy stream, overlapping compute.
//  * Each request's arithmetic depends only on its matrix, its partitions,
//    its x and its passes, and every tick but a request's last runs whole
//    blocks of 8 of its steps, so its passes do not depend on the load: its
//    results are the same alone and in any mix.
// One scheduler serves three drivers: msrep_serve replays a trace known in
// advance on the GPU; msrep_server_* runs the scheduler on a thread of its
// own and takes requests as they come (submit / poll); msrep_serve_simulate
// replays a trace against a simulated device on a virtual clock, for testing
// on a CPU.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <type_traits>
#include <vector>

#include "batched.hpp"

namespace msrep {
namespace {

constexpr int kRing = 4;     // tick events in rotation (at most kInflight ticks in flight)
constexpr int kInflight = 2;
constexpr int64_t kDefaultQueue = int64_t(1) << 20;  // incremental server's waiting requests
constexpr int32_t kMaxStepsPerTick = 64;
constexpr int32_t kDefaultStepsPerTick = kMaxStepsPerTick;
constexpr int64_t kTickRounds = 1;  // a tick's items: at most this many rounds of resident waves
// passes (of at most 8 columns) that k steps of a request take in a tick
constexpr int32_t pass_count(int32_t k) { return (k + kSpmmMaxCols - 1) / kSpmmMaxCols; }

// ------------------------------------------------------- tick descriptors
// A request slot of the server: its resident matrix, partitions, carries and
// vectors.  A request's steps that share a tick are the columns of a
// multi-vector product, stored in blocks of ld = min(8, copies) columns: block
// b of X is n x ld row-major at X + b*n*ld, of Y m x ld at Y + b*m*ld; column c
// (step j0 + c of the tick) is column c % ld of block c / ld, and its head and
// tail carries sit at carry + c*2*np.  Written once when the request is
// admitted.
struct ServeSlot {
  BatchMat M;
  BatchXY xy;
  int64_t rid;
  int32_t ld;     // columns per block of X and Y
  int32_t ebytes; // bytes of an x or y element
};

constexpr int kTickMax = 240;  // requests per tick (the arguments stay below 4 KB)

// One serving tick: an entry per request it runs (its slot; its first step
// j0 and its count k of steps, as j0 | k << 16) and two prefix sums over the
// entries: of their partition counts (the merge's items: (request,
// partition)), and of partitions times passes (the product's items:
// (request, partition, pass), pass b covering columns 8b .. 8b+7).  Passed
// by value as kernel arguments.
struct TickSrc {
  const ServeSlot *table;
  int64_t n_items, n_pass_items;
  int32_t n_waves, count;
  int32_t slot[kTickMax];
  int32_t step[kTickMax];  // j0 | k << 16
  int32_t begin[kTickMax + 1];
  int32_t pbegin[kTickMax + 1];
  __device__ static int32_t first_of(int32_t v) { return v & 0xffff; }
  __device__ static int32_t count_of(int32_t v) { return v >> 16; }
  // the entry i with b[i] <= it < b[i+1]
  __device__ int32_t find(const int32_t *b, int64_t it) const {
    int32_t lo = 0, hi = count;
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (b[mid] <= it)
        lo = mid;
      else
        hi = mid;
    }
    return lo;
  }
  __device__ int32_t entry_of(int64_t it) const { return find(begin, it); }
  // equal item counts per group (a request's partitions hold equal
  // nonzeros, so items cost about the same)
  __device__ void group(int32_t g, int32_t G, int64_t &lo, int64_t &hi) const {
    lo = n_items * g / G;
    hi = n_items * (g + 1) / G;
  }
};

// The tick's (request, partition) items seen by the boundary merge for column
// blockIdx.y: a request running fewer steps has no such column (m = 0:
// nothing written).
struct TickColSrc : TickSrc {
  __device__ void get(int64_t it, BItem &o) const {
    const int32_t i = entry_of(it);
    const ServeSlot *S = table + slot[i];
    bitem_from(S->M, S->xy, static_cast<int32_t>(it - begin[i]), o);
    const int32_t c = static_cast<int32_t>(blockIdx.y), ld = S->ld;
    o.ldy = ld;
    if (c < count_of(step[i])) {
      o.y = static_cast<char *>(o.y) +
            (static_cast<int64_t>(c / ld) * S->M.m * ld + c % ld) * S->ebytes;
      o.carry += static_cast<int64_t>(c) * 2 * S->M.np;
    } else {
      o.m = 0;
    }
  }
};

// a tick's descriptor and the merge's alpha and beta fit the 4 KB of
// kernel arguments
static_assert(sizeof(TickColSrc) + 2 * sizeof(double) <= 4096, "tick arguments above 4 KB");

// The tick's products: resident wavefronts, those of one XCD sweeping its
// group of (request, partition, pass) items together (a partition's passes
// are neighbours, so they read its slice of A through one L2).  Pass b of a
// request running k steps covers columns 8b .. min(k, 8b+8) - 1 of block b:
// one 8-column pass of the multi-vector routine, or passes of 4, 2 and 1.
// Every request's passes depend only on its own k, so its arithmetic does
// not depend on the tick's other requests.
template <int VT>
__global__ __launch_bounds__(kSpmmWaves * kWave) __attribute__((amdgpu_waves_per_eu(4))) void
serve_passes(const TickSrc src) {
  using Tr = vt_traits<VT>;
  using T = typename Tr::T;
  using V = typename Tr::V;
  __shared__ int32_t s_mark_all[kSpmmWaves][kWave];
  __shared__ int32_t s_rows_all[kSpmmWaves][kWave];
  const int wid = threadIdx.x / kWave;
  const int wpb = blockDim.x / kWave;
  const int nb = static_cast<int>(gridDim.x);
  const int G = nb < kXcds ? nb : kXcds;
  const int g = static_cast<int>(blockIdx.x) % G;
  const int j = (static_cast<int>(blockIdx.x) / G) * wpb + wid;
  const int wg = (nb / G + (g < nb % G ? 1 : 0)) * wpb;
  const int64_t lo = src.n_pass_items * g / G, hi = src.n_pass_items * (g + 1) / G;
  for (int64_t it = lo + j; it < hi; it += wg) {
    const int32_t i = uniform(src.find(src.pbegin, it));
    const ServeSlot *S = src.table + src.slot[i];
    const int32_t k = TickSrc::count_of(src.step[i]);
    const int32_t passes = pass_count(k);
    const int32_t li = static_cast<int32_t>(it - src.pbegin[i]);
    const int32_t p = li / passes, blk = li % passes;
    const int32_t *col = uniform(S->M.col);
    const V *val = static_cast<const V *>(uniform(S->M.val));
    const msrep_part *parts = uniform(S->M.parts);
    const int32_t *lptr = uniform(S->M.lptr);
    const int32_t m = uniform(S->M.m), n = uniform(S->M.n), np = uniform(S->M.np);
    const int64_t ld = uniform(S->ld);
    const int64_t cs = 2 * static_cast<int64_t>(np);
    // the pass's block of X, Y and carries
    const T *X = static_cast<const T *>(uniform(S->xy.x)) + blk * static_cast<int64_t>(n) * ld;
    T *Y = static_cast<T *>(uniform(S->xy.y)) + blk * static_cast<int64_t>(m) * ld;
    double *carry = uniform(S->M.carry) + static_cast<int64_t>(blk) * kSpmmMaxCols * cs;
    const int32_t w = min(kSpmmMaxCols, k - blk * kSpmmMaxCols);  // columns of this pass
    int32_t c0 = 0;
    auto pass = [&](auto nr_c, auto cpl_c) {
      constexpr int NR = decltype(nr_c)::value, CPL = decltype(cpl_c)::value;
      // bytes from the pass's first column to the end of the block of X and of Y
      const int64_t xe = static_cast<int64_t>(n) * ld - c0, ye = static_cast<int64_t>(m) * ld - c0;
      const uint32_t xb = static_cast<uint32_t>((xe > 0 ? xe : 0) * sizeof(T));
      const uint32_t yb = static_cast<uint32_t>((ye > 0 ? ye : 0) * sizeof(T));
      spmm_partition<VT, NR, true, CPL>(col, val, parts, lptr, np, p, X + c0, ld, Y + c0, ld, m,
                                        1.0, 0.0, carry + c0 * cs, cs, xb, yb, s_mark_all[wid],
                                        s_rows_all[wid]);
      c0 += NR;
      wave_lds_sync();
    };
    if (w == 8) pass(std::integral_constant<int, 8>{}, std::integral_constant<int, 2>{});
    if (w - c0 >= 4) pass(std::integral_constant<int, 4>{}, std::integral_constant<int, 1>{});
    if (w - c0 >= 2) pass(std::integral_constant<int, 2>{}, std::integral_constant<int, 1>{});
    if (w - c0 >= 1) pass(std::integral_constant<int, 1>{}, std::integral_constant<int, 1>{});
  }
}

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

// X of every request of a tick: block row i fills entry i's k columns, column
// c (column c % ld of block c / ld) with x of step j0 + c.
template <typename T>
__global__ void fill_x_tick(const TickSrc src, uint64_t seed) {
  const ServeSlot *S = src.table + src.slot[blockIdx.y];
  const int32_t sc = src.step[blockIdx.y];
  T *X = static_cast<T *>(const_cast<void *>(S->xy.x));
  const int32_t n = S->M.n, j0 = TickSrc::first_of(sc), k = TickSrc::count_of(sc);
  const int64_t rid = S->rid, ld = S->ld;
  for (int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; c < n;
       c += int64_t(gridDim.x) * blockDim.x)
    for (int32_t s = 0; s < k; ++s)
      X[(s / ld) * n * ld + c * ld + s % ld] = static_cast<T>(x_value(seed, rid, j0 + s, c));
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
enum State { kWaiting, kLoading, kReady, kDraining, kDone };

struct Resident {  // a pool matrix in the arena, with its partitions
  bool present = false;
  size_t off = 0, bytes = 0;
  int32_t np = 1;         // partitions, shared by every request on the matrix
  int refs = 0;
  int64_t last_use = 0;
  double ready_at = 0;   // simulated executor
  hipEvent_t ev{};       // HIP executor: upload finished
};

struct Req {
  int64_t key = 0;        // trace index (replay) or submission number (server)
  msrep_request r{};
  void *y_host = nullptr; // last y copied here when it finishes (optional)
  State st = kWaiting;
  int32_t np = 1, slot = -1;
  int32_t copies = 1;         // columns of X and Y: steps one tick may run
  int32_t last_copy = 0;      // the column the last step ran in
  // columns per block of X and Y, and blocks
  int32_t ld() const { return copies < kSpmmMaxCols ? copies : kSpmmMaxCols; }
  int32_t blocks() const { return (copies + ld() - 1) / ld(); }
  size_t off = 0, bytes = 0;  // X, Y, carries
  size_t x_off = 0, y_off = 0, carry_off = 0;
  int32_t enq = 0;            // steps enqueued
  int64_t last_tick = -1;
  double t_arrive = 0, t_admit = 0, t_done = 0, ready_at = 0;
  hipEvent_t ev{};            // partitions and descriptor in place
};

struct Completion {
  int64_t key, rid;
  double t_arrive, t_admit, t_done;
  msrep_status status;
  int32_t matrix, steps;
};

// A resident matrix's region: its arrays (ptr, idx, val; what is uploaded),
// then its partitions and local pointers (built on the device after the
// upload, once for every request on the matrix).
size_t mat_array_bytes(const msrep_mat &A) {
  return align_up(4 * (static_cast<size_t>(A.m) + 1), 256) +
         align_up(4 * static_cast<size_t>(A.nnz), 256) +
         align_up(static_cast<size_t>(value_bytes(A.vtype)) * A.nnz, 256);
}
size_t part_bytes(int32_t np) { return align_up(sizeof(msrep_part) * static_cast<size_t>(np), 256); }
size_t mat_bytes(const msrep_mat &A, int32_t np) {
  return mat_array_bytes(A) + part_bytes(np) +
         align_up(4 * static_cast<size_t>(msrep_lptr_bound(A.m, np)), 256);
}

void layout_req(Req &q, const msrep_mat &A) {
  const size_t xb = vec_bytes(A.vtype);
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o += align_up(b ? b : 1, 256);
    return at;
  };
  const size_t c = static_cast<size_t>(q.copies);
  const size_t cb = static_cast<size_t>(q.ld()) * q.blocks();  // whole blocks
  q.x_off = take(xb * static_cast<size_t>(A.n) * cb);
  q.y_off = take(xb * static_cast<size_t>(A.m) * cb);
  q.carry_off = take(16 * static_cast<size_t>(q.np) * c);
  q.bytes = o;
}

// k consecutive steps of one request in a tick, from step j0.
struct Entry {
  Req *q;
  int32_t j0, k;
};

struct Tick {
  int64_t id;
  std::vector<Entry> ent;
  int32_t requests = 0;
  double end = 0;  // simulated
};

// ------------------------------------------------------- HIP executor
struct HipExec {
  const msrep_serve_cfg &cfg;
  const msrep_host_mat *pool;
  char *arena;
  hipStream_t copy{}, comp{};
  hipEvent_t t0{};
  hipEvent_t tick_ev[kRing]{};
  std::vector<hipEvent_t> ev_free;  // recycled per-request and per-matrix events
  std::chrono::steady_clock::time_point w0;
  int32_t vtype, max_slots = 0;
  size_t table_off = 0;
  ServeSlot *slots_h = nullptr;  // pinned staging of the slot table
  int n_waves_max = 0;
  int64_t wave_slots() const { return n_waves_max; }

  HipExec(const msrep_serve_cfg &c, const msrep_host_mat *p, int32_t vt)
      : cfg(c), pool(p), arena(static_cast<char *>(c.arena_d)), vtype(vt) {}

  size_t table_bytes() const { return align_up(sizeof(ServeSlot) * max_slots, 256); }

  msrep_status init(Arena &A, int32_t slots) {
    max_slots = slots;
    MSREP_HIP(hipStreamCreateWithFlags(&copy, hipStreamNonBlocking));
    MSREP_HIP(hipStreamCreateWithFlags(&comp, hipStreamNonBlocking));
    MSREP_HIP(hipEventCreate(&t0));
    for (auto &e : tick_ev) MSREP_HIP(hipEventCreate(&e));
    if (!A.alloc(table_bytes(), &table_off))
      return fail(MSREP_ERR_BUDGET, "msrep_serve: budget too small for the slot table");
    MSREP_HIP(hipHostMalloc(reinterpret_cast<void **>(&slots_h), table_bytes()));
    std::memset(slots_h, 0, table_bytes());
    int dev = 0, per_cu = 0;
    hipDeviceProp_t prop;
    MSREP_HIP(hipGetDevice(&dev));
    MSREP_HIP(hipGetDeviceProperties(&prop, dev));
    if (vtype == MSREP_F64)
      MSREP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, serve_passes<MSREP_F64>, kSpmmWaves * kWave, 0));
    else
      MSREP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, serve_passes<MSREP_F32>, kSpmmWaves * kWave, 0));
    n_waves_max = std::max(1, per_cu) * kSpmmWaves * prop.multiProcessorCount;
    MSREP_HIP(hipEventRecord(t0, comp));
    MSREP_HIP(hipEventSynchronize(t0));
    w0 = std::chrono::steady_clock::now();
    return MSREP_OK;
  }
  size_t reserved_bytes() const { return table_bytes(); }
  void shutdown() {
    if (copy) (void)hipStreamSynchronize(copy);
    if (comp) (void)hipStreamSynchronize(comp);
    if (slots_h) (void)hipHostFree(slots_h);
    slots_h = nullptr;
    for (auto &e : tick_ev)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : ev_free) (void)hipEventDestroy(e);
    ev_free.clear();
    if (t0) (void)hipEventDestroy(t0);
    if (copy) (void)hipStreamDestroy(copy);
    if (comp) (void)hipStreamDestroy(comp);
    t0 = nullptr;
    copy = comp = nullptr;
  }
  double now() const {
    const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - w0).count();
    return s * cfg.time_scale;
  }
  msrep_status take_event(hipEvent_t *e) {
    if (*e) return MSREP_OK;
    if (!ev_free.empty()) {
      *e = ev_free.back();
      ev_free.pop_back();
      return MSREP_OK;
    }
    MSREP_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
    return MSREP_OK;
  }
  void give_event(hipEvent_t *e) {
    if (*e) ev_free.push_back(*e);
    *e = nullptr;
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
  msrep_part *res_parts(int32_t k, const Resident &R) const {
    return reinterpret_cast<msrep_part *>(arena + R.off + mat_array_bytes(pool[k].A));
  }
  int32_t *res_lptr(int32_t k, const Resident &R) const {
    return reinterpret_cast<int32_t *>(arena + R.off + mat_array_bytes(pool[k].A) +
                                       part_bytes(R.np));
  }
  // The matrix's arrays, then its partitions, on the copy stream.
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
    if (msrep_status st = msrep_build_partition(&D, R.np, res_parts(k, R), res_lptr(k, R),
                                                msrep_lptr_bound(D.m, R.np), nullptr, copy))
      return st;
    if (msrep_status st = take_event(&R.ev)) return st;
    MSREP_HIP(hipEventRecord(R.ev, copy));
    return MSREP_OK;
  }
  void evicted(Resident &R) { give_event(&R.ev); }
  // The request's slot descriptor (its matrix's partitions, its own vectors
  // and carries), on the copy stream after the matrix upload.
  msrep_status prepare(Req &q, const Resident &R) {
    const msrep_mat D = device_mat(q.r.matrix, R);
    char *b = arena + q.off;
    ServeSlot &S = slots_h[q.slot];
    S.M = BatchMat{D.idx, D.val, res_parts(q.r.matrix, R), res_lptr(q.r.matrix, R), D.m, D.n,
                   R.np, 0, reinterpret_cast<double *>(b + q.carry_off)};
    S.xy = BatchXY{b + q.x_off, b + q.y_off};
    S.rid = q.r.rid;
    S.ld = q.ld();
    S.ebytes = static_cast<int32_t>(vec_bytes(D.vtype));
    // the slot was last read by ticks that completed before it was freed
    MSREP_HIP(hipMemcpyAsync(arena + table_off + sizeof(ServeSlot) * q.slot, &S, sizeof(ServeSlot),
                             hipMemcpyHostToDevice, copy));
    if (msrep_status st = take_event(&q.ev)) return st;
    MSREP_HIP(hipEventRecord(q.ev, copy));
    return MSREP_OK;
  }
  bool ready(Req &q) { return hipEventQuery(q.ev) == hipSuccess; }
  void released(Req &q) { give_event(&q.ev); }

  msrep_status launch(Tick &t, const std::vector<Resident> &) {
    TickSrc src;
    src.table = reinterpret_cast<const ServeSlot *>(arena + table_off);
    src.count = static_cast<int32_t>(t.ent.size());
    int64_t items = 0, pitems = 0;
    int32_t max_n = 1, kmax = 1;
    for (int32_t i = 0; i < src.count; ++i) {
      const Entry &e = t.ent[i];
      const Req &q = *e.q;
      src.slot[i] = q.slot;
      src.step[i] = e.j0 | (e.k << 16);
      src.begin[i] = static_cast<int32_t>(items);
      src.pbegin[i] = static_cast<int32_t>(pitems);
      items += q.np;
      pitems += static_cast<int64_t>(q.np) * pass_count(e.k);
      max_n = std::max(max_n, pool[q.r.matrix].A.n);
      kmax = std::max(kmax, e.k);
    }
    src.begin[src.count] = static_cast<int32_t>(items);
    src.pbegin[src.count] = static_cast<int32_t>(pitems);
    src.n_items = items;
    src.n_pass_items = pitems;
    src.n_waves = static_cast<int32_t>(std::min<int64_t>(n_waves_max, std::max<int64_t>(1, pitems)));
    TickColSrc msrc;
    static_cast<TickSrc &>(msrc) = src;
    const int grid = (src.n_waves + kSpmmWaves - 1) / kSpmmWaves;
    const int gm = static_cast<int>((items + kMergeBlock - 1) / kMergeBlock);
    // x fill: a thread per row of X up to about 8192 blocks in all, so that a
    // lone request's fill spreads over the chip
    const int fill_x = std::min((max_n + 255) / 256, std::max(64, 8192 / src.count));
    const dim3 gf(static_cast<unsigned>(fill_x), static_cast<unsigned>(src.count));
    const dim3 gmc(static_cast<unsigned>(gm > 0 ? gm : 1), static_cast<unsigned>(kmax));
    if (vtype == MSREP_F64) {
      hipLaunchKernelGGL(fill_x_tick<double>, gf, dim3(256), 0, comp, src, cfg.seed);
      hipLaunchKernelGGL(serve_passes<MSREP_F64>, dim3(grid), dim3(kSpmmWaves * kWave), 0, comp,
                         src);
      hipLaunchKernelGGL((merge_items<double, true, TickColSrc>), gmc, dim3(kMergeBlock), 0, comp,
                         msrc, 1.0, 0.0);
    } else {
      hipLaunchKernelGGL(fill_x_tick<float>, gf, dim3(256), 0, comp, src, cfg.seed);
      hipLaunchKernelGGL(serve_passes<MSREP_F32>, dim3(grid), dim3(kSpmmWaves * kWave), 0, comp,
                         src);
      hipLaunchKernelGGL((merge_items<float, true, TickColSrc>), gmc, dim3(kMergeBlock), 0, comp,
                         msrc, 1.0, 0.0);
    }
    MSREP_LAUNCHED("serve tick");
    MSREP_HIP(hipEventRecord(tick_ev[t.id % kRing], comp));
    return MSREP_OK;
  }
  bool done(Tick &t, double *at) {
    hipEvent_t e = tick_ev[t.id % kRing];
    if (hipEventQuery(e) != hipSuccess) return false;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, t0, e);
    *at = ms * 1e-3 * cfg.time_scale;
    return true;
  }
  msrep_status keep_y(Req &q) {
    if (!q.y_host) return MSREP_OK;
    const msrep_mat &H = pool[q.r.matrix].A;
    // column last_copy of the request's Y: column last_copy % ld of block
    // last_copy / ld (m rows of ld values)
    const size_t eb = vec_bytes(vtype), ld = static_cast<size_t>(q.ld());
    const size_t at = (q.last_copy / ld) * ld * static_cast<size_t>(H.m) + q.last_copy % ld;
    MSREP_HIP(hipMemcpy2D(q.y_host, eb, arena + q.off + q.y_off + eb * at, eb * ld, eb,
                          static_cast<size_t>(H.m), hipMemcpyDeviceToHost));
    return MSREP_OK;
  }
  // Nothing to do: spin while the device works, else sleep until the next
  // arrival (at most 200 us, so that a late event is not missed for long).
  void idle(double until, bool busy) {
    const double wait = until - now();
    if (busy || wait <= 0) {
      std::this_thread::yield();
      return;
    }
    // a sleep overshoots by up to the timer slack (tens of microseconds):
    // sleep until shortly before the next arrival and spin the rest
    const double s = std::min(wait / cfg.time_scale, 2e-4) - 8e-5;
    if (s > 0)
      std::this_thread::sleep_for(std::chrono::duration<double>(s));
    else
      std::this_thread::yield();
  }
  void release_all(std::vector<Resident> &res) {
    for (auto &r : res) give_event(&r.ev);
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
  int64_t wave_slots() const { return 4096; }
  msrep_status init(Arena &, int32_t) { return MSREP_OK; }
  size_t reserved_bytes() const { return 0; }
  void shutdown() {}
  double now() const { return clock; }
  msrep_status upload(int32_t k, Resident &R) {
    copy_free = std::max(copy_free, clock) + static_cast<double>(mat_array_bytes(pool[k].A)) / upload_bw;
    R.ready_at = copy_free;
    return MSREP_OK;
  }
  void evicted(Resident &) {}
  msrep_status prepare(Req &q, const Resident &R) {
    copy_free = std::max({copy_free, clock, R.ready_at}) + 5e-6;
    q.ready_at = copy_free;
    return MSREP_OK;
  }
  bool ready(Req &q) { return clock >= q.ready_at; }
  void released(Req &) {}
  msrep_status launch(Tick &t, const std::vector<Resident> &) {
    double work = tick_cost;
    for (const Entry &e : t.ent)
      work += 2.0 * e.k * static_cast<double>(pool[e.q->r.matrix].A.nnz) / flop_rate;
    dev_free = std::max(dev_free, clock) + work;
    t.end = dev_free;
    return MSREP_OK;
  }
  bool done(Tick &t, double *at) {
    if (clock < t.end) return false;
    *at = t.end;
    return true;
  }
  msrep_status keep_y(Req &) { return MSREP_OK; }
  // advance the virtual clock to the next thing that can happen
  double next_event = 0;
  void idle(double until, bool) { clock = std::max(clock, std::min(until, next_event)); }
  void release_all(std::vector<Resident> &) {}
};

// ------------------------------------------------------------ scheduler
// Admission, residency, eviction and tick formation, independent of how
// requests arrive and how the device is driven.
template <class Exec>
class Scheduler {
 public:
  Scheduler(Exec &ex, const msrep_serve_cfg &cfg, const msrep_host_mat *pool, int32_t pool_size)
      : ex_(ex), cfg_(cfg), pool_(pool), pool_size_(pool_size), arena_(cfg.budget_bytes),
        res_(pool_size) {}

  msrep_status init() {
    if (msrep_status st = ex_.init(arena_, cfg_.max_slots)) return st;
    for (int32_t s = cfg_.max_slots - 1; s >= 0; --s) free_slots_.push_back(s);
    return MSREP_OK;
  }
  int32_t np_of(int32_t k) const {
    const msrep_host_mat &H = pool_[k];
    const int64_t npw = std::max(1, cfg_.nnz_per_wave);
    return H.np > 0 ? H.np : static_cast<int32_t>(std::max<int64_t>(1, (H.A.nnz + npw - 1) / npw));
  }
  // More pool matrices (the incremental server's registrations): pool
  // points at the whole pool, the first pool_size_ entries unchanged.
  void grow_pool(const msrep_host_mat *pool, int32_t pool_size) {
    pool_ = pool;
    pool_size_ = pool_size;
    res_.resize(static_cast<size_t>(pool_size));
  }
  int32_t steps_per_tick() const {
    return cfg_.steps_per_tick > 0 ? cfg_.steps_per_tick : kDefaultStepsPerTick;
  }
  // Steps of request q in a tick whose cap is `cap` (a multiple of 8): all
  // that are left if they fit, else whole blocks of 8.  Every tick but a
  // request's last so runs a multiple of 8 of its steps, its passes are the
  // same whatever the caps were, and so are its results (with fewer than 8
  // copies, steps_per_tick below 8, a tick runs up to `copies` steps).
  static int32_t steps_this_tick(const Req &q, int32_t cap) {
    const int32_t left = q.r.steps - q.enq;
    if (q.copies < kSpmmMaxCols) return std::min(q.copies, left);
    const int32_t lim = std::min(q.copies, cap);
    return left <= lim ? left : lim / kSpmmMaxCols * kSpmmMaxCols;
  }
  // A request arrives (at q->t_arrive on the scheduler's clock).
  void arrive(std::unique_ptr<Req> q) {
    q->np = np_of(q->r.matrix);
    q->copies = std::max(1, std::min(steps_per_tick(), q->r.steps));
    // a tick's (partition, pass) items of one request stay below 2^31
    const int64_t max_pass = ((int64_t(1) << 31) - 1) / q->np;
    if (pass_count(q->copies) > max_pass)
      q->copies = static_cast<int32_t>(max_pass * kSpmmMaxCols);
    layout_req(*q, pool_[q->r.matrix].A);
    // a request whose vectors would hold more than a sixteenth of the arena
    // reserves 8 columns (what a tick under load runs), so that a small
    // arena still holds many requests; its results are the same
    if (q->copies > kSpmmMaxCols && q->bytes > arena_.cap() / 16) {
      q->copies = kSpmmMaxCols;
      layout_req(*q, pool_[q->r.matrix].A);
    }
    q->st = kWaiting;
    waiting_.push_back(q.get());
    owned_.push_back(std::move(q));
  }
  // Device work the host must watch: ticks in flight, or requests whose
  // uploads and partitions are being prepared (the host launches their
  // first tick as soon as those are done).
  bool device_busy() const {
    if (!inflight_.empty()) return true;
    for (const Req *q : admitted_)
      if (q->st == kLoading) return true;
    return false;
  }
  bool empty() const { return waiting_.empty() && admitted_.empty() && inflight_.empty(); }
  size_t waiting() const { return waiting_.size(); }
  // The earliest time something in flight can change (simulated executor).
  double next_event(double until) const {
    double nx = until;
    for (const Tick &t : inflight_) nx = std::min(nx, t.end);
    for (Req *q : admitted_)
      if (q->st == kLoading) nx = std::min(nx, q->ready_at);
    return nx;
  }

  // One pass: admit, mark loaded requests ready, retire finished ticks,
  // launch the next tick.  Returns whether anything happened.
  bool step(msrep_status &err) {
    const double now = ex_.now();
    bool progressed = admit(now, err);
    if (err) return progressed;
    for (Req *q : admitted_)
      if (q->st == kLoading && ex_.ready(*q)) {
        q->st = kReady;
        progressed = true;
      }
    while (!inflight_.empty()) {
      double at = 0;
      if (!ex_.done(inflight_.front(), &at)) break;
      Tick &t = inflight_.front();
      for (const Entry &e : t.ent) {
        Req *q = e.q;
        if (e.j0 + e.k == q->r.steps) {  // the request's last steps: once per request
          if (msrep_status st = ex_.keep_y(*q)) err = st;
          finish(*q, MSREP_OK, at);
          res_[q->r.matrix].refs--;
          res_[q->r.matrix].last_use = ++use_clock_;
          arena_.release(q->off);
          free_slots_.push_back(q->slot);
          ex_.released(*q);
        }
      }
      inflight_.pop_front();
      admitted_.erase(std::remove_if(admitted_.begin(), admitted_.end(),
                                     [](Req *q) { return q->st == kDone; }),
                      admitted_.end());
      progressed = true;
    }
    if (err) return progressed;
    if (static_cast<int>(inflight_.size()) < kInflight) {
      Tick t;
      t.id = tick_id_;
      // ready requests taken round robin over the admitted list, so that
      // none waits more than one tick for a turn (kTickMax requests a tick)
      const size_t na = admitted_.size();
      take_.clear();
      for (size_t j = 0; j < na && static_cast<int>(take_.size()) < kTickMax; ++j) {
        Req *q = admitted_[(rr_ + j) % na];
        if (q->st == kReady && q->enq < q->r.steps) take_.push_back(q);
      }
      // the most steps of a request in this tick: the largest multiple of 8
      // that keeps the tick's (partition, pass) items within kTickRounds
      // rounds of the resident wavefronts.  A lone request then runs all its
      // steps in a tick or two; a busy server runs 8 of each, so that each
      // request's matrix is read once per tick and the x blocks the tick
      // gathers from stay few.
      const int64_t room = kTickRounds * ex_.wave_slots();
      int32_t cap = kSpmmMaxCols;
      for (int32_t c = kMaxStepsPerTick; c > kSpmmMaxCols; c -= kSpmmMaxCols) {
        int64_t items = 0;
        for (const Req *q : take_)
          items += static_cast<int64_t>(q->np) * pass_count(steps_this_tick(*q, c));
        if (items <= room) {
          cap = c;
          break;
        }
      }
      // (partition, pass) items below 2^31 in all
      int64_t pitems = 0;
      for (Req *q : take_) {
        const int32_t k = steps_this_tick(*q, cap);
        pitems += static_cast<int64_t>(q->np) * pass_count(k);
        if (pitems >= (int64_t(1) << 31)) break;
        t.ent.push_back(Entry{q, q->enq, k});
      }
      if (na) rr_ = (rr_ + t.ent.size()) % na;
      if (!t.ent.empty()) {
        t.requests = static_cast<int32_t>(t.ent.size());
        peak_active_ = std::max(peak_active_, t.requests);
        if (msrep_status st = ex_.launch(t, res_)) {
          err = st;
          return progressed;
        }
        for (const Entry &e : t.ent) {
          Req *q = e.q;
          q->enq = e.j0 + e.k;
          q->last_tick = t.id;
          q->last_copy = e.k - 1;
          if (q->enq == q->r.steps) q->st = kDraining;
        }
        inflight_.push_back(std::move(t));
        ++tick_id_;
        ++ticks_;
        progressed = true;
      }
    }
    return progressed;
  }

  // Completions since the last call (their Req records are freed).
  std::vector<Completion> take_completed() {
    std::vector<Completion> out;
    out.swap(done_);
    owned_.erase(std::remove_if(owned_.begin(), owned_.end(),
                                [](const std::unique_ptr<Req> &q) { return q->st == kDone; }),
                 owned_.end());
    return out;
  }
  void shutdown() {
    ex_.shutdown();
    ex_.release_all(res_);
  }
  int64_t ticks() const { return ticks_; }
  int32_t peak_active() const { return peak_active_; }
  size_t peak_bytes() const { return arena_.peak(); }

 private:
  void finish(Req &q, msrep_status st, double t) {
    q.st = kDone;
    q.t_done = t;
    done_.push_back(Completion{q.key, q.r.rid, q.t_arrive, q.t_admit, t, st, q.r.matrix,
                               q.r.steps});
  }
  // first come, first served
  bool admit(double now, msrep_status &err) {
    bool progressed = false;
    while (!waiting_.empty() && !free_slots_.empty()) {
      Req &q = *waiting_.front();
      Resident &R = res_[q.r.matrix];
      const size_t mb = mat_bytes(pool_[q.r.matrix].A, q.np);
      const size_t table = std::min(arena_.cap(), ex_.reserved_bytes());
      if (q.bytes + mb + 512 > arena_.cap() - table) {  // can never fit
        waiting_.pop_front();
        finish(q, MSREP_ERR_BUDGET, now);
        progressed = true;
        continue;
      }
      // make room: evict idle resident matrices, least recently used first
      bool got = false;
      for (;;) {
        size_t mo = 0, ro = 0;
        const bool need_mat = !R.present;
        bool ok_mat = true;
        if (need_mat) ok_mat = arena_.alloc(mb, &mo);
        const bool ok_req = ok_mat && arena_.alloc(q.bytes, &ro);
        if (ok_mat && ok_req) {
          if (need_mat) {
            R.present = true;
            R.off = mo;
            R.bytes = mb;
            R.np = q.np;
            if (msrep_status st = ex_.upload(q.r.matrix, R)) {
              err = st;
              return progressed;
            }
          }
          q.off = ro;
          got = true;
          break;
        }
        if (ok_mat && need_mat) arena_.release(mo);
        int32_t victim = -1;
        for (int32_t k = 0; k < pool_size_; ++k)
          if (res_[k].present && res_[k].refs == 0 && k != q.r.matrix &&
              (victim < 0 || res_[k].last_use < res_[victim].last_use))
            victim = k;
        if (victim < 0) break;
        arena_.release(res_[victim].off);
        res_[victim].present = false;
        ex_.evicted(res_[victim]);
      }
      if (!got) break;  // wait for running requests to free memory
      R.refs++;
      R.last_use = ++use_clock_;
      q.slot = free_slots_.back();
      free_slots_.pop_back();
      if (msrep_status st = ex_.prepare(q, R)) {
        err = st;
        return progressed;
      }
      q.st = kLoading;
      q.t_admit = now;
      waiting_.pop_front();
      admitted_.push_back(&q);
      progressed = true;
    }
    return progressed;
  }

  Exec &ex_;
  std::vector<Req *> take_;  // the requests a tick takes
  const msrep_serve_cfg &cfg_;
  const msrep_host_mat *pool_;
  int32_t pool_size_;
  Arena arena_;
  std::vector<Resident> res_;
  std::vector<std::unique_ptr<Req>> owned_;
  std::deque<Req *> waiting_;
  std::vector<Req *> admitted_;  // loading, ready or draining
  std::deque<Tick> inflight_;
  std::vector<int32_t> free_slots_;
  std::vector<Completion> done_;
  int64_t tick_id_ = 0, ticks_ = 0, use_clock_ = 0;
  size_t rr_ = 0;
  int32_t peak_active_ = 0;
};

// Latency statistics over completions.
void fill_stats(const std::vector<Completion> &all, const msrep_host_mat *pool, int64_t ticks,
                int32_t peak_active, size_t peak_bytes, msrep_serve_stats *stats) {
  if (!stats) return;
  std::vector<double> lat;
  double first = 1e300, last = 0, flops = 0;
  int64_t steps = 0, failed = 0;
  for (const Completion &c : all) {
    first = std::min(first, c.t_arrive);
    if (c.status != MSREP_OK) {
      ++failed;
      continue;
    }
    lat.push_back((c.t_done - c.t_arrive) * 1e3);
    last = std::max(last, c.t_done);
    steps += c.steps;
    flops += 2.0 * static_cast<double>(pool[c.matrix].A.nnz) * c.steps;
  }
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
  stats->peak_bytes = static_cast<int64_t>(peak_bytes);
  stats->peak_active = peak_active;
}

// Replay of a trace known in advance: requests arrive at their trace times.
template <class Exec>
msrep_status replay(Exec &ex, const msrep_serve_cfg &cfg, const msrep_host_mat *pool,
                    int32_t pool_size, const msrep_request *trace, int64_t n_req,
                    msrep_result *results, msrep_serve_stats *stats) {
  Scheduler<Exec> sch(ex, cfg, pool, pool_size);
  if (msrep_status st = sch.init()) {
    sch.shutdown();
    return st;
  }
  std::vector<int64_t> order(n_req);
  for (int64_t i = 0; i < n_req; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return trace[a].t_arrive < trace[b].t_arrive; });
  std::vector<Completion> all;
  all.reserve(n_req);
  int64_t next = 0;
  msrep_status err = MSREP_OK;
  while (static_cast<int64_t>(all.size()) < n_req && err == MSREP_OK) {
    const double now = ex.now();
    bool progressed = false;
    while (next < n_req && trace[order[next]].t_arrive <= now) {
      const int64_t i = order[next++];
      auto q = std::make_unique<Req>();
      q->key = i;
      q->r = trace[i];
      q->t_arrive = trace[i].t_arrive;
      q->y_host = cfg.keep_y ? results[i].y_host : nullptr;
      sch.arrive(std::move(q));
      progressed = true;
    }
    progressed |= sch.step(err);
    for (const Completion &c : sch.take_completed()) {
      msrep_result &r = results[c.key];
      r.t_arrive = c.t_arrive;
      r.t_admit = c.t_admit;
      r.t_done = c.t_done;
      r.status = c.status;
      all.push_back(c);
    }
    if (!progressed && err == MSREP_OK) {
      const double until = next < n_req ? trace[order[next]].t_arrive : now + 1.0;
      if constexpr (std::is_same_v<Exec, SimExec>) ex.next_event = sch.next_event(until);
      ex.idle(until, sch.device_busy());
    }
  }
  sch.shutdown();
  if (err) return err;
  fill_stats(all, pool, sch.ticks(), sch.peak_active(), sch.peak_bytes(), stats);
  return ok();
}

// One pool matrix: CSR of the pool's value type, a supported shape, and
// host arrays (when it will be uploaded).
msrep_status check_pool_mat(const msrep_host_mat &H, int32_t vt, bool need_arrays,
                            const char *who, int32_t k) {
  const msrep_mat &A = H.A;
  if (A.fmt != MSREP_CSR || A.vtype != vt)
    return fail(MSREP_ERR_ARG, "%s: pool matrix %d must be CSR of the pool's value type", who, k);
  // (a block of 8 columns of a request's X or Y stays below 4 GiB)
  if (A.m < 0 || A.n < 0 || A.nnz < 0 || A.nnz >= (int64_t(1) << 31) || A.n >= (1 << 24) ||
      A.m >= (1 << 26) || H.np < 0)
    return fail(MSREP_ERR_ARG, "%s: pool matrix %d has an unsupported shape", who, k);
  if (need_arrays && (!A.ptr || (A.nnz > 0 && (!A.idx || !A.val))))
    return fail(MSREP_ERR_ARG, "%s: pool matrix %d has NULL arrays", who, k);
  return MSREP_OK;
}

msrep_status check_cfg_pool(const msrep_serve_cfg *cfg, const msrep_host_mat *pool,
                            int32_t pool_size, bool need_arena, const char *who) {
  if (!cfg || !pool || pool_size <= 0)
    return fail(MSREP_ERR_ARG, "%s: missing configuration or pool", who);
  if (need_arena && !cfg->arena_d) return fail(MSREP_ERR_ARG, "%s: arena_d is NULL", who);
  if (cfg->max_slots < 1 || cfg->max_slots > 4096)
    return fail(MSREP_ERR_ARG, "%s: max_slots must be 1..4096", who);
  if (!(cfg->time_scale > 0)) return fail(MSREP_ERR_ARG, "%s: time_scale must be > 0", who);
  if (cfg->max_queue < 0) return fail(MSREP_ERR_ARG, "%s: max_queue must be >= 0", who);
  if (cfg->steps_per_tick < 0 || cfg->steps_per_tick > kMaxStepsPerTick)
    return fail(MSREP_ERR_ARG, "%s: steps_per_tick must be 0..%d", who, kMaxStepsPerTick);
  const int32_t vt = pool[0].A.vtype;
  if (vt != MSREP_F64 && vt != MSREP_F32)
    return fail(MSREP_ERR_UNSUPPORTED, "%s: pool matrices must be F64 or F32", who);
  for (int32_t k = 0; k < pool_size; ++k)
    if (msrep_status st = check_pool_mat(pool[k], vt, need_arena, who, k)) return st;
  return MSREP_OK;
}

msrep_status check_request(const msrep_request &r, int32_t pool_size, const char *who,
                           long long i) {
  if (r.matrix < 0 || r.matrix >= pool_size || r.steps < 1 || r.steps > 65535 || r.rid < 0 ||
      r.rid >= (int64_t(1) << 24))
    return fail(MSREP_ERR_ARG, "%s: request %lld is malformed", who, i);
  return MSREP_OK;
}

msrep_status check_serve_args(const msrep_serve_cfg *cfg, const msrep_host_mat *pool,
                              int32_t pool_size, const msrep_request *trace, int64_t n_req,
                              msrep_result *results, bool need_arena) {
  if (n_req < 0 || (n_req > 0 && (!trace || !results)))
    return fail(MSREP_ERR_ARG, "msrep_serve: missing trace or results");
  if (msrep_status st = check_cfg_pool(cfg, pool, pool_size, need_arena, "msrep_serve")) return st;
  for (int64_t i = 0; i < n_req; ++i)
    if (msrep_status st = check_request(trace[i], pool_size, "msrep_serve", i)) return st;
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
  return replay(ex, *cfg, pool, pool_size, trace, n_req, results, stats);
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
  return replay(ex, *cfg, pool, pool_size, trace, n_req, results, stats);
}

// ------------------------------------------------------ incremental server
// The scheduler on a thread of its own; submit() hands requests over through
// an inbox, completions come back through an outbox that poll() drains.
struct msrep_server_s {
  msrep_serve_cfg cfg{};
  std::vector<msrep_host_mat> pool;     // the worker's pool (registrations applied)
  std::vector<msrep_host_mat> pending;  // registered, not yet applied (under mu)
  int32_t pool_count = 0;               // pool + pending: valid matrix indices (under mu)
  int32_t vtype = 0;                    // the pool's value type (fixed at creation)
  int device = 0;
  std::unique_ptr<HipExec> ex;
  std::unique_ptr<Scheduler<HipExec>> sch;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_in, cv_out;
  std::deque<std::unique_ptr<Req>> inbox;
  std::deque<Completion> outbox;
  std::vector<Completion> all;  // every completion, for the final statistics
  int64_t submitted = 0, waiting = 0;  // waiting: admission queue (inbox not included)
  bool stop = false;
  msrep_status err = MSREP_OK;
  std::string err_text;

  void run() {
    (void)hipSetDevice(device);
    for (;;) {
      std::vector<std::unique_ptr<Req>> in;
      std::vector<msrep_host_mat> reg;
      bool stopping;
      {
        std::lock_guard<std::mutex> lk(mu);
        while (!inbox.empty()) {
          in.push_back(std::move(inbox.front()));
          inbox.pop_front();
        }
        reg.swap(pending);
        stopping = stop;
      }
      if (!reg.empty()) {  // before the requests, which may name the new matrices
        pool.insert(pool.end(), reg.begin(), reg.end());
        ex->pool = pool.data();
        sch->grow_pool(pool.data(), static_cast<int32_t>(pool.size()));
      }
      for (auto &q : in) {
        q->t_arrive = ex->now();
        sch->arrive(std::move(q));
      }
      msrep_status e = MSREP_OK;
      bool progressed = sch->step(e) || !in.empty();
      std::vector<Completion> c = sch->take_completed();
      if (!c.empty() || e) {
        std::lock_guard<std::mutex> lk(mu);
        for (const Completion &x : c) {
          outbox.push_back(x);
          all.push_back(x);
        }
        waiting = static_cast<int64_t>(sch->waiting());
        if (e) {
          err = e;
          err_text = last_error();
        }
      } else {
        std::lock_guard<std::mutex> lk(mu);
        waiting = static_cast<int64_t>(sch->waiting());
      }
      if (!c.empty() || e) cv_out.notify_all();
      if (e) break;
      if (stopping && sch->empty()) {
        std::lock_guard<std::mutex> lk(mu);
        if (inbox.empty()) break;
        continue;
      }
      if (!progressed) {
        if (sch->device_busy()) {
          std::this_thread::yield();
        } else {
          std::unique_lock<std::mutex> lk(mu);
          cv_in.wait_for(lk, std::chrono::microseconds(200),
                         [&] { return !inbox.empty() || stop; });
        }
      }
    }
    cv_out.notify_all();
  }
};

extern "C" msrep_status msrep_server_create(const msrep_serve_cfg *cfg, const msrep_host_mat *pool,
                                            int32_t pool_size, msrep_server *out) {
  const char *who = "msrep_server_create";
  if (!out) return fail(MSREP_ERR_ARG, "%s: out is NULL", who);
  *out = nullptr;
  if (msrep_status st = check_cfg_pool(cfg, pool, pool_size, true, who)) return st;
  auto s = std::make_unique<msrep_server_s>();
  s->cfg = *cfg;
  s->pool.assign(pool, pool + pool_size);
  s->pool_count = pool_size;
  s->vtype = pool[0].A.vtype;
  MSREP_HIP(hipGetDevice(&s->device));
  s->ex = std::make_unique<HipExec>(s->cfg, s->pool.data(), pool[0].A.vtype);
  s->sch = std::make_unique<Scheduler<HipExec>>(*s->ex, s->cfg, s->pool.data(), pool_size);
  if (msrep_status st = s->sch->init()) {
    s->sch->shutdown();
    return st;
  }
  msrep_server_s *raw = s.get();
  try {
    s->worker = std::thread([raw] { raw->run(); });
  } catch (...) {
    s->sch->shutdown();
    return fail(MSREP_ERR_ARG, "%s: cannot start the scheduler thread", who);
  }
  *out = s.release();
  return ok();
}

extern "C" msrep_status msrep_server_submit(msrep_server s, const msrep_request *req,
                                            void *y_host) {
  const char *who = "msrep_server_submit";
  if (!s || !req) return fail(MSREP_ERR_ARG, "%s: server or request is NULL", who);
  auto q = std::make_unique<Req>();
  q->r = *req;
  q->y_host = y_host;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (msrep_status st = check_request(*req, s->pool_count, who, 0)) return st;
    if (s->err) return fail(s->err, "%s: the server stopped: %s", who, s->err_text.c_str());
    if (s->stop) return fail(MSREP_ERR_ARG, "%s: the server is being destroyed", who);
    const int64_t cap = s->cfg.max_queue > 0 ? s->cfg.max_queue : kDefaultQueue;
    if (s->waiting + static_cast<int64_t>(s->inbox.size()) >= cap)
      return fail(MSREP_ERR_BUSY, "%s: %lld requests already wait", who,
                  static_cast<long long>(cap));
    q->key = s->submitted++;
    s->inbox.push_back(std::move(q));
  }
  s->cv_in.notify_one();
  return ok();
}

extern "C" msrep_status msrep_server_register(msrep_server s, const msrep_host_mat *mat,
                                              int32_t *index) {
  const char *who = "msrep_server_register";
  if (!s || !mat || !index) return fail(MSREP_ERR_ARG, "%s: server, matrix or index is NULL", who);
  *index = -1;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (msrep_status st = check_pool_mat(*mat, s->vtype, true, who, s->pool_count))
      return st;
    if (s->err) return fail(s->err, "%s: the server stopped: %s", who, s->err_text.c_str());
    if (s->stop) return fail(MSREP_ERR_ARG, "%s: the server is being destroyed", who);
    if (s->pool_count == INT32_MAX) return fail(MSREP_ERR_SIZE, "%s: the pool is full", who);
    s->pending.push_back(*mat);
    *index = s->pool_count++;
  }
  s->cv_in.notify_one();
  return ok();
}

extern "C" int64_t msrep_server_poll(msrep_server s, msrep_completion *out, int64_t cap,
                                     int32_t timeout_ms) {
  if (!s || (cap > 0 && !out) || cap < 0)
    return fail(MSREP_ERR_ARG, "msrep_server_poll: server or output is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->outbox.empty() && timeout_ms > 0 && !s->err)
    s->cv_out.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                       [&] { return !s->outbox.empty() || s->err; });
  int64_t n = 0;
  while (n < cap && !s->outbox.empty()) {
    const Completion &c = s->outbox.front();
    out[n++] = msrep_completion{c.rid, c.t_arrive, c.t_admit, c.t_done, c.status, 0};
    s->outbox.pop_front();
  }
  if (n == 0 && s->err) return fail(s->err, "msrep_server_poll: %s", s->err_text.c_str());
  return n;
}

extern "C" msrep_status msrep_server_destroy(msrep_server s, msrep_serve_stats *stats) {
  if (!s) return ok();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_in.notify_all();
  if (s->worker.joinable()) s->worker.join();
  s->sch->shutdown();
  const msrep_status err = s->err;
  const std::string text = s->err_text;
  fill_stats(s->all, s->pool.data(), s->sch->ticks(), s->sch->peak_active(), s->sch->peak_bytes(),
             stats);
  delete s;
  if (err) return fail(err, "msrep_server_destroy: the server had stopped: %s", text.c_str());
  return ok();
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
