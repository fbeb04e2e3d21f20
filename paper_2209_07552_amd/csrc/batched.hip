// Batched SpMV: y_k = alpha*A_k*x_k + beta*y_k for many CSR matrices in one
// persistent launch, captured once in a hipGraph.
//
// Each matrix is split into its own equal-nnz partitions (msRep
// Algorithm 2).  All partitions of all matrices form one work list; the host
// cuts the list into contiguous runs of about equal nonzero count, one run
// per resident wavefront (the same equal-nnz rule, applied across the whole
// batch), so no queue or atomic is needed and a wavefront keeps working on
// one matrix for long stretches.  A second kernel completes the rows split
// between partitions, for every matrix at once.
#include <algorithm>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "batched.hpp"

namespace msrep {

msrep_status resolve_tune(const msrep_tune *tune, int *K, int *wpb, int *pf, int *resident,
                          const char *who);

namespace {

constexpr int kDefaultNnzPerWave = 1024;
constexpr int kMaxWaves = 16384;

int64_t nnz_per_wave_of(const msrep_tune *tunes, int32_t k) {
  const int v = tunes ? tunes[k].nnz_per_wave : 0;
  return v > 0 ? v : kDefaultNnzPerWave;
}

int32_t parts_of(const msrep_mat &A, int64_t npw) {
  const int64_t np = (A.nnz + npw - 1) / npw;
  return static_cast<int32_t>(np < 1 ? 1 : np);
}

struct Layout {
  std::vector<size_t> parts_off, lptr_off;
  size_t items_off, groups_off, mats_off, xy_off, carry_off, total;
  int64_t n_items;
};

Layout layout(int32_t count, const msrep_mat *mats, const msrep_tune *tunes) {
  Layout L;
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o += align_up(b, 256);
    return at;
  };
  L.n_items = 0;
  for (int32_t k = 0; k < count; ++k) {
    const int32_t np = parts_of(mats[k], nnz_per_wave_of(tunes, k));
    L.parts_off.push_back(take(sizeof(msrep_part) * static_cast<size_t>(np)));
    L.lptr_off.push_back(take(4 * static_cast<size_t>(msrep_lptr_bound(mats[k].m, np))));
    L.n_items += np;
  }
  L.items_off = take(sizeof(int2) * static_cast<size_t>(L.n_items));
  L.groups_off = take(sizeof(int64_t) * (kXcds + 1));
  L.mats_off = take(sizeof(BatchMat) * static_cast<size_t>(count));
  L.xy_off = take(sizeof(BatchXY) * static_cast<size_t>(count));
  L.carry_off = take(16 * static_cast<size_t>(L.n_items));
  L.total = o;
  return L;
}

}  // namespace
}  // namespace msrep

using namespace msrep;

struct msrep_plan_s {
  int32_t count = 0, vtype = 0, K = 4, wpb = 4, pf = 1, n_waves = 0, grid = 0;
  int64_t n_items = 0;
  char *ws = nullptr;
  Layout L;
  BatchXY *xy_d = nullptr;
  BatchXY *staging = nullptr;  // pinned host copy of the x/y table
  hipEvent_t staged{};
  hipEvent_t done{};  // after the last graph launch (it reads xy_d and the carries)
  hipStream_t cap{};
  hipGraph_t graph{};
  hipGraphExec_t exec{};
  int device = 0;
};

extern "C" size_t msrep_plan_ws_bytes(int32_t count, const msrep_mat *mats,
                                      const msrep_tune *tunes) {
  if (count <= 0 || !mats) return 0;
  return layout(count, mats, tunes).total;
}

extern "C" int64_t msrep_plan_items(msrep_plan plan) { return plan ? plan->n_items : 0; }

extern "C" msrep_status msrep_plan_destroy(msrep_plan plan) {
  if (!plan) return ok();
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  if (plan->cap) (void)hipStreamDestroy(plan->cap);
  if (plan->staged) (void)hipEventDestroy(plan->staged);
  if (plan->done) (void)hipEventDestroy(plan->done);
  if (plan->staging) (void)hipHostFree(plan->staging);
  delete plan;
  return ok();
}

namespace {

template <int VT, int K, bool B0, int PF>
msrep_status capture_kernels(msrep_plan P, double alpha, double beta) {
  using T = typename vt_traits<VT>::T;
  PlanSrc src;
  src.mats = reinterpret_cast<const BatchMat *>(P->ws + P->L.mats_off);
  src.xy = P->xy_d;
  src.items = reinterpret_cast<const int2 *>(P->ws + P->L.items_off);
  src.group_begin = reinterpret_cast<const int64_t *>(P->ws + P->L.groups_off);
  src.n_items = P->n_items;
  src.n_waves = P->n_waves;
  src._pad = 0;
  const size_t lds = seg_lds_per_wave<VT, K>() * P->wpb;
  hipLaunchKernelGGL((spmv_items_persistent<VT, K, B0, PF, PlanSrc>), dim3(P->grid),
                     dim3(P->wpb * kWave), lds, P->cap, src, alpha, beta);
  MSREP_LAUNCHED("spmv_batched_persistent");
  const int g = static_cast<int>((P->n_items + kMergeBlock - 1) / kMergeBlock);
  hipLaunchKernelGGL((merge_items<T, B0, PlanSrc>), dim3(g > 0 ? g : 1), dim3(kMergeBlock), 0,
                     P->cap, src, alpha, beta);
  MSREP_LAUNCHED("merge_batched");
  return MSREP_OK;
}

template <int VT>
msrep_status capture_vt(msrep_plan P, double alpha, double beta) {
  const bool b0 = beta == 0.0;
  if (P->pf == 2) {
    if (P->K == 8)
      return b0 ? capture_kernels<VT, 8, true, 2>(P, alpha, beta)
                : capture_kernels<VT, 8, false, 2>(P, alpha, beta);
    return b0 ? capture_kernels<VT, 4, true, 2>(P, alpha, beta)
              : capture_kernels<VT, 4, false, 2>(P, alpha, beta);
  }
  if (P->K == 8)
    return b0 ? capture_kernels<VT, 8, true, 1>(P, alpha, beta)
              : capture_kernels<VT, 8, false, 1>(P, alpha, beta);
  return b0 ? capture_kernels<VT, 4, true, 1>(P, alpha, beta)
            : capture_kernels<VT, 4, false, 1>(P, alpha, beta);
}

template <int VT, int K, int PF>
int resident_blocks(int wpb) {
  int nb = 0;
  const size_t lds = seg_lds_per_wave<VT, K>() * wpb;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, spmv_items_persistent<VT, K, true, PF, PlanSrc>, wpb * kWave, lds) != hipSuccess)
    return 0;
  return nb;
}

template <int VT>
int resident_vt(int K, int pf, int wpb) {
  if (pf == 2) return K == 8 ? resident_blocks<VT, 8, 2>(wpb) : resident_blocks<VT, 4, 2>(wpb);
  return K == 8 ? resident_blocks<VT, 8, 1>(wpb) : resident_blocks<VT, 4, 1>(wpb);
}

int resident_for(int32_t vtype, int K, int pf, int wpb) {
  switch (vtype) {
    case MSREP_F64: return resident_vt<MSREP_F64>(K, pf, wpb);
    case MSREP_F32: return resident_vt<MSREP_F32>(K, pf, wpb);
    default: return resident_vt<MSREP_BF16>(K, pf, wpb);
  }
}

}  // namespace

extern "C" msrep_status msrep_plan_create(int32_t count, const msrep_mat *mats,
                                          const msrep_tune *tunes, double alpha, double beta,
                                          void *ws_d, size_t ws_bytes, void *stream,
                                          msrep_plan *out) {
  if (!out) return fail(MSREP_ERR_ARG, "msrep_plan_create: out is NULL");
  *out = nullptr;
  if (count <= 0 || !mats) return fail(MSREP_ERR_ARG, "msrep_plan_create: no matrices");
  for (int32_t k = 0; k < count; ++k) {
    if (msrep_status st = check_mat(&mats[k], "msrep_plan_create")) return st;
    if (mats[k].fmt != MSREP_CSR)
      return fail(MSREP_ERR_UNSUPPORTED, "msrep_plan_create: matrix %d is not CSR", k);
    if (mats[k].vtype != mats[0].vtype)
      return fail(MSREP_ERR_ARG, "msrep_plan_create: matrices must share one value type");
    if (static_cast<uint64_t>(mats[k].n) * vec_bytes(mats[k].vtype) >= (uint64_t(1) << 32))
      return fail(MSREP_ERR_UNSUPPORTED, "msrep_plan_create: x of matrix %d exceeds 4 GiB", k);
  }
  int K, wpb, pf, resident;  // (the batched kernel's grid is always resident)
  if (msrep_status st = resolve_tune(tunes, &K, &wpb, &pf, &resident, "msrep_plan_create"))
    return st;
  Layout L = layout(count, mats, tunes);
  if (!ws_d || ws_bytes < L.total)
    return fail(MSREP_ERR_SIZE, "msrep_plan_create: workspace of %zu bytes needed (got %zu)",
                L.total, ws_d ? ws_bytes : size_t(0));
  hipStream_t s = as_stream(stream);
  auto P = new msrep_plan_s();
  P->count = count;
  P->vtype = mats[0].vtype;
  P->K = K;
  P->wpb = wpb;
  // loads one chunk ahead unless the tune asks for two (more registers)
  P->pf = tunes && tunes[0].pipeline == 2 ? 2 : 1;
  P->ws = static_cast<char *>(ws_d);
  P->L = L;
  P->n_items = L.n_items;
  auto bail = [&](msrep_status st) {
    msrep_plan_destroy(P);
    return st;
  };
  if (hipGetDevice(&P->device) != hipSuccess) return bail(fail(MSREP_ERR_HIP, "hipGetDevice"));
  // partitions of every matrix, built on the device
  std::vector<BatchMat> bm(count);
  std::vector<int2> items;
  std::vector<int64_t> item_nnz;
  items.reserve(L.n_items);
  item_nnz.reserve(L.n_items);
  for (int32_t k = 0; k < count; ++k) {
    const msrep_mat &A = mats[k];
    const int32_t np = parts_of(A, nnz_per_wave_of(tunes, k));
    msrep_part *parts = reinterpret_cast<msrep_part *>(P->ws + L.parts_off[k]);
    int32_t *lptr = reinterpret_cast<int32_t *>(P->ws + L.lptr_off[k]);
    if (msrep_status st = msrep_build_partition(&A, np, parts, lptr, msrep_lptr_bound(A.m, np),
                                                nullptr, stream))
      return bail(st);
    double *carry = reinterpret_cast<double *>(P->ws + L.carry_off) + 2 * static_cast<int64_t>(items.size());
    bm[k] = BatchMat{A.idx, A.val, parts, lptr, A.m, A.n, np, 0, carry};
    for (int32_t p = 0; p < np; ++p) {
      items.push_back(int2{k, p});
      item_nnz.push_back(item_cost(A.nnz, A.m, np, p));
    }
  }
  // resident wavefronts; the items in equal-work groups, one per XCD
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, P->device) != hipSuccess)
    return bail(fail(MSREP_ERR_HIP, "hipGetDeviceProperties"));
  int per_cu = resident_for(P->vtype, K, P->pf, wpb);
  if (per_cu < 1) per_cu = 1;
  int64_t waves = static_cast<int64_t>(per_cu) * wpb * prop.multiProcessorCount;
  waves = std::min<int64_t>({waves, kMaxWaves, std::max<int64_t>(1, L.n_items)});
  P->grid = static_cast<int>((waves + wpb - 1) / wpb);
  P->n_waves = static_cast<int32_t>(waves);
  const int32_t groups = std::min<int32_t>(kXcds, P->grid);
  std::vector<int64_t> wb(groups + 1, L.n_items);
  equal_work_runs(item_nnz.data(), L.n_items, groups, wb.data());
  P->xy_d = reinterpret_cast<BatchXY *>(P->ws + L.xy_off);
  if (hipMemcpyAsync(P->ws + L.items_off, items.data(), sizeof(int2) * items.size(),
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(P->ws + L.groups_off, wb.data(), sizeof(int64_t) * wb.size(),
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(P->ws + L.mats_off, bm.data(), sizeof(BatchMat) * bm.size(),
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return bail(fail(MSREP_ERR_HIP, "msrep_plan_create: upload of the plan tables failed"));
  if (hipHostMalloc(reinterpret_cast<void **>(&P->staging), sizeof(BatchXY) * count) != hipSuccess)
    return bail(fail(MSREP_ERR_HIP, "msrep_plan_create: hipHostMalloc failed"));
  std::memset(P->staging, 0, sizeof(BatchXY) * count);
  if (hipEventCreateWithFlags(&P->staged, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(P->staged, s) != hipSuccess ||
      hipEventCreateWithFlags(&P->done, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(P->done, s) != hipSuccess)
    return bail(fail(MSREP_ERR_HIP, "msrep_plan_create: event setup failed"));
  // capture the two launches once
  if (hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(MSREP_ERR_HIP, "msrep_plan_create: stream creation failed"));
  if (hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return bail(fail(MSREP_ERR_HIP, "msrep_plan_create: hipStreamBeginCapture failed"));
  msrep_status st;
  switch (P->vtype) {
    case MSREP_F64: st = capture_vt<MSREP_F64>(P, alpha, beta); break;
    case MSREP_F32: st = capture_vt<MSREP_F32>(P, alpha, beta); break;
    default: st = capture_vt<MSREP_BF16>(P, alpha, beta);
  }
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(P->cap, &g);
  if (st) {
    if (g) (void)hipGraphDestroy(g);
    return bail(st);
  }
  if (ec != hipSuccess || !g) return bail(fail(MSREP_ERR_HIP, "msrep_plan_create: capture failed"));
  P->graph = g;
  if (hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0) != hipSuccess)
    return bail(fail(MSREP_ERR_HIP, "msrep_plan_create: hipGraphInstantiate failed"));
  *out = P;
  return ok();
}

extern "C" msrep_status msrep_spmv_batched(msrep_plan plan, const void *const *x_ptrs,
                                           void *const *y_ptrs, void *stream) {
  if (!plan) return fail(MSREP_ERR_ARG, "msrep_spmv_batched: plan is NULL");
  if (!x_ptrs || !y_ptrs) return fail(MSREP_ERR_ARG, "msrep_spmv_batched: x/y arrays are NULL");
  hipStream_t s = as_stream(stream);
  // the previous call's copy out of the staging table must be done
  MSREP_HIP(hipEventSynchronize(plan->staged));
  for (int32_t k = 0; k < plan->count; ++k) {
    plan->staging[k].x = x_ptrs[k];
    plan->staging[k].y = y_ptrs[k];
  }
  // the previous launch, on whatever stream, still reads xy_d and the
  // carries: the rewrite waits for it on the device
  MSREP_HIP(hipStreamWaitEvent(s, plan->done, 0));
  MSREP_HIP(hipMemcpyAsync(plan->xy_d, plan->staging, sizeof(BatchXY) * plan->count,
                           hipMemcpyHostToDevice, s));
  MSREP_HIP(hipEventRecord(plan->staged, s));
  MSREP_HIP(hipGraphLaunch(plan->exec, s));
  MSREP_HIP(hipEventRecord(plan->done, s));
  return ok();
}
