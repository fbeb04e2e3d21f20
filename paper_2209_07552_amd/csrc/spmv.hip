// msrep_spmv: dispatch of the per-format SpMV kernels and of the boundary
// merge, plus the shared C-ABI helpers (errors, descriptor checks).
#include <map>
#include <mutex>
#include <tuple>

#include "common.hpp"
#include "spmv_coo.hpp"
#include "spmv_csc.hpp"
#include "spmv_cscw.hpp"
#include "spmv_csr.hpp"

namespace msrep {

std::string &last_error() {
  static thread_local std::string e;
  return e;
}

msrep_status fail(msrep_status code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  last_error() = buf;
  return code;
}

int value_bytes(int32_t vtype) {
  switch (vtype) {
    case MSREP_F64: return 8;
    case MSREP_F32: return 4;
    case MSREP_BF16: return 2;
    default: return 0;
  }
}

msrep_status check_mat(const msrep_mat *A, const char *who) {
  if (!A) return fail(MSREP_ERR_ARG, "%s: matrix descriptor is NULL", who);
  if (A->fmt < MSREP_CSR || A->fmt > MSREP_COO_COL)
    return fail(MSREP_ERR_ARG, "%s: unknown format %d", who, A->fmt);
  if (!value_bytes(A->vtype)) return fail(MSREP_ERR_ARG, "%s: unknown value type %d", who, A->vtype);
  if (A->m < 0 || A->n < 0 || A->nnz < 0)
    return fail(MSREP_ERR_ARG, "%s: negative size (m=%d n=%d nnz=%lld)", who, A->m, A->n,
                static_cast<long long>(A->nnz));
  if (A->nnz >= (int64_t(1) << 31))
    return fail(MSREP_ERR_SIZE, "%s: nnz=%lld does not fit int32 indices", who,
                static_cast<long long>(A->nnz));
  if (A->nnz > 0 && (A->m == 0 || A->n == 0))
    return fail(MSREP_ERR_ARG, "%s: nonzeros in a matrix with no rows or columns", who);
  const bool coo = A->fmt == MSREP_COO || A->fmt == MSREP_COO_ANY || A->fmt == MSREP_COO_COL;
  if (!coo && !A->ptr) return fail(MSREP_ERR_ARG, "%s: ptr is NULL", who);
  if (A->nnz > 0 && (!A->idx || !A->val)) return fail(MSREP_ERR_ARG, "%s: idx/val is NULL", who);
  if (coo && A->nnz > 0 && !A->idx2)
    return fail(MSREP_ERR_ARG, "%s: COO col_idx (idx2) is NULL", who);
  return MSREP_OK;
}

namespace {

// Blocks of `threads` threads (dyn_lds bytes of LDS each) that the device
// holds at once, capped at want; cached per kernel, shape and device.
template <typename Kern>
int resident_grid(Kern kernel, int threads, size_t dyn_lds, int64_t want) {
  static std::mutex mu;
  static std::map<std::tuple<const void *, int, size_t, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  const auto key = std::make_tuple(reinterpret_cast<const void *>(kernel), threads, dyn_lds, dev);
  int g;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) {
      g = it->second;
    } else {
      int per_cu = 0, cus = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, dyn_lds) !=
          hipSuccess)
        per_cu = 1;
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 1;
      g = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
      cache.emplace(key, g);
    }
  }
  return static_cast<int>(want < g ? (want > 0 ? want : 1) : g);
}

template <int VT, int K, bool B0>
msrep_status launch_csr(const msrep_mat *A, const msrep_part *parts, const int32_t *lptr,
                        int32_t np, const void *x, void *y, double alpha, double beta, int wpb,
                        int pf, int resident, double *carry, hipStream_t s) {
  using Tr = vt_traits<VT>;
  const size_t lds = seg_lds_per_wave<VT, K>() * wpb;
  const int64_t want = (np + wpb - 1) / wpb;  // one wavefront per partition
  timing_begin("spmv_csr_seg", s);
  if (pf == 1)
    hipLaunchKernelGGL((spmv_csr_seg<VT, K, B0, 1>),
                       dim3(resident ? resident_grid(spmv_csr_seg<VT, K, B0, 1>, wpb * kWave, lds, want)
                                : want),
                       dim3(wpb * kWave), lds, s, A->idx,
                       static_cast<const typename Tr::V *>(A->val), parts, lptr, np,
                       static_cast<const typename Tr::T *>(x), static_cast<typename Tr::T *>(y),
                       A->m, A->n, alpha, beta, carry);
  else
    hipLaunchKernelGGL((spmv_csr_seg<VT, K, B0, 2>),
                       dim3(resident ? resident_grid(spmv_csr_seg<VT, K, B0, 2>, wpb * kWave, lds, want)
                                : want),
                       dim3(wpb * kWave), lds, s, A->idx,
                       static_cast<const typename Tr::V *>(A->val), parts, lptr, np,
                       static_cast<const typename Tr::T *>(x), static_cast<typename Tr::T *>(y),
                       A->m, A->n, alpha, beta, carry);
  MSREP_LAUNCHED("spmv_csr_seg");
  timing_end("spmv_csr_seg", s);
  return MSREP_OK;
}

template <int VT, int K, bool B0>
msrep_status launch_coo(const msrep_mat *A, const msrep_part *parts, int32_t np, const void *x,
                        void *y, double alpha, double beta, int wpb, int resident, double *carry,
                        hipStream_t s) {
  using Tr = vt_traits<VT>;
  const size_t lds = coo_lds_per_wave<VT, K>() * wpb;
  const int64_t want = (np + wpb - 1) / wpb;  // one wavefront per partition
  timing_begin("spmv_coo_seg", s);
  hipLaunchKernelGGL((spmv_coo_seg<VT, K, B0>),
                     dim3(resident ? resident_grid(spmv_coo_seg<VT, K, B0>, wpb * kWave, lds, want)
                                   : want),
                     dim3(wpb * kWave), lds, s, A->idx, A->idx2,
                     static_cast<const typename Tr::V *>(A->val), A->nnz, parts, np,
                     static_cast<const typename Tr::T *>(x), static_cast<typename Tr::T *>(y),
                     A->m, A->n, alpha, beta, carry);
  MSREP_LAUNCHED("spmv_coo_seg");
  timing_end("spmv_coo_seg", s);
  return MSREP_OK;
}

constexpr int kPhaseAll = 0, kPhaseStructure = 1, kPhaseNumeric = 2;

// The structure-only kernels of the CSC path: per-bucket counts of every
// producer, their scan into run offsets, and the bucket pieces.  They depend
// on A's row indices, the partitions and np, not on x or the values.
msrep_status csc_structure(const msrep_mat *A, const msrep_part *parts, int32_t np,
                           const CscLayout &L, char *b, hipStream_t s) {
  int32_t *cnt = reinterpret_cast<int32_t *>(b + L.cnt);
  int32_t *agg = reinterpret_cast<int32_t *>(b + L.agg);
  int32_t *pbase = reinterpret_cast<int32_t *>(b + L.pbase);
  int32_t *mbase = reinterpret_cast<int32_t *>(b + L.mbase);
  int32_t *mlist = reinterpret_cast<int32_t *>(b + L.mlist);
  const size_t cur_lds = align_up(static_cast<size_t>(L.nb) * 4, 16);
  timing_begin("csc_count", s);
  hipLaunchKernelGGL(csc_count, dim3(L.P), dim3(kCscScatterWaves * kWave), cur_lds, s, A->idx,
                     A->nnz, parts, np, L.P, A->m, L.shift, L.nb, cnt);
  MSREP_LAUNCHED("csc_count");
  timing_end("csc_count", s);
  timing_begin("csc_scan", s);
  if (msrep_status st = scan::device_scan<int32_t, scan::SumOp>(
          cnt, cnt, static_cast<int64_t>(L.nb) * L.P + 1, agg, false, s))
    return st;
  timing_end("csc_scan", s);
  timing_begin("csc_plan", s);
  hipLaunchKernelGGL(csc_plan, dim3(1), dim3(kPlanBlock), 0, s, cnt, L.nb, L.P, L.piece, pbase,
                     mbase, mlist);
  MSREP_LAUNCHED("csc_plan");
  timing_end("csc_plan", s);
  return MSREP_OK;
}

// PACK: one record per product (msrep_tune.pipeline == 1), else value and
// row-offset arrays.  phase: kPhaseAll, kPhaseStructure (csc_structure only)
// or kPhaseNumeric (the workspace already holds csc_structure's output).
template <int VT, int K, bool PACK>
msrep_status launch_csc(const msrep_mat *A, const msrep_part *parts, const int32_t *lptr,
                        int32_t np, const void *x, void *y, double alpha, double beta, int wpb,
                        void *ws, int phase, hipStream_t s) {
  using Tr = vt_traits<VT>;
  using T = typename Tr::T;
  using Acc = typename Tr::A;
  CscLayout L;
  if (!csc_layout(A->m, A->nnz, np, sizeof(Acc), L))
    return fail(MSREP_ERR_UNSUPPORTED, "msrep_spmv: CSC supports at most %d rows",
                kCscMaxBuckets << kCscMaxShift);
  char *b = static_cast<char *>(ws);
  if (phase != kPhaseNumeric)
    if (msrep_status st = csc_structure(A, parts, np, L, b, s)) return st;
  if (phase == kPhaseStructure) return MSREP_OK;
  int32_t *cnt = reinterpret_cast<int32_t *>(b + L.cnt);
  int32_t *pbase = reinterpret_cast<int32_t *>(b + L.pbase);
  int32_t *mbase = reinterpret_cast<int32_t *>(b + L.mbase);
  int32_t *mlist = reinterpret_cast<int32_t *>(b + L.mlist);
  Acc *prod = reinterpret_cast<Acc *>(b + L.prod);
  uint16_t *rlo = reinterpret_cast<uint16_t *>(b + L.rlo);
  double *part = reinterpret_cast<double *>(b + L.part);
  (void)wpb;  // the scatter always runs 16-wavefront producers
  timing_begin("csc_scatter", s);
  if (A->fmt == MSREP_COO_ANY || A->fmt == MSREP_COO_COL)  // columns read from col_idx
    hipLaunchKernelGGL((coo_any_scatter<VT, K, PACK>), dim3(L.P), dim3(kCscScatterWaves * kWave),
                       align_up((static_cast<size_t>(L.nb) + kWave) * 4, 16), s, A->idx, A->idx2,
                       static_cast<const typename Tr::V *>(A->val), A->nnz, parts, np, L.P,
                       static_cast<const T *>(x), A->m, A->n, L.shift, L.nb, cnt, prod, rlo);
  else
    hipLaunchKernelGGL((csc_scatter<VT, K, PACK>), dim3(L.P), dim3(kCscScatterWaves * kWave),
                       csc_scatter_lds<K>(L.nb), s, A->idx,
                       static_cast<const typename Tr::V *>(A->val), A->nnz, parts, lptr, np, L.P,
                       static_cast<const T *>(x), A->m, A->n, L.shift, L.nb, cnt, prod, rlo);
  MSREP_LAUNCHED("csc_scatter");
  timing_end("csc_scatter", s);
  timing_begin("csc_reduce", s);
  hipLaunchKernelGGL((csc_reduce<T, Acc, PACK>), dim3(static_cast<uint32_t>(L.max_pieces)),
                     dim3(kReduceBlock), sizeof(double) << L.shift, s, prod, rlo, cnt, pbase, mbase,
                     L.nb, L.P, L.shift, A->m, A->nnz, L.piece, L.max_slots, part, static_cast<T *>(y),
                     alpha, beta);
  MSREP_LAUNCHED("csc_reduce");
  timing_end("csc_reduce", s);
  timing_begin("csc_merge", s);
  {
    // buckets of several pieces hold more than L.piece products each
    const int64_t most = std::min<int64_t>(L.nb, A->nnz / L.piece + 1);
    const int64_t blocks = std::min<int64_t>(most * ((1 << L.shift) / kCscBlock), 2048);
    hipLaunchKernelGGL((csc_merge<T>), dim3(static_cast<uint32_t>(blocks > 0 ? blocks : 1)),
                       dim3(kCscBlock), 0, s, pbase, mbase, mlist, L.nb, L.shift, A->m,
                       L.max_slots, part, static_cast<T *>(y), alpha, beta);
  }
  MSREP_LAUNCHED("csc_merge");
  timing_end("csc_merge", s);
  return MSREP_OK;
}

// The windowed CSC path (spmv_cscw.hpp): its numeric regions overlap the
// bucketed products, its structure regions follow both (cscw_layout).
void cscw_place(const msrep_mat *A, int32_t np, const CscLayout &L, CscwLayout &W) {
  cscw_layout(A->m, A->nnz, np, L, W);
}

msrep_status cscw_structure(const msrep_mat *A, const msrep_part *parts, int32_t np,
                            const CscwLayout &W, char *b, hipStream_t s) {
  int32_t *wlist = reinterpret_cast<int32_t *>(b + W.wlist);
  int32_t *wcnt = reinterpret_cast<int32_t *>(b + W.wcnt);
  int32_t *flags = reinterpret_cast<int32_t *>(b + W.flags);
  int32_t *inv_cnt = reinterpret_cast<int32_t *>(b + W.inv_cnt);
  int32_t *inv_off = reinterpret_cast<int32_t *>(b + W.inv_off);
  int32_t *inv_agg = reinterpret_cast<int32_t *>(b + W.inv_agg);
  int32_t *inv_list = reinterpret_cast<int32_t *>(b + W.inv_list);
  timing_begin("cscw_windows", s);
  hipLaunchKernelGGL(cscw_fill_i32, dim3(static_cast<unsigned>(std::min<int64_t>((W.nwin + 256) / 256, 4096))),
                     dim3(256), 0, s, inv_cnt, W.nwin + 1, int32_t(0));
  hipLaunchKernelGGL(cscw_fill_i32, dim3(1), dim3(64), 0, s, flags, int64_t(4), int32_t(0));
  hipLaunchKernelGGL(cscw_windows, dim3(W.P), dim3(1024), 0, s, A->idx, A->nnz, parts, np, W.P,
                     A->m, wlist, wcnt, flags, inv_cnt);
  MSREP_LAUNCHED("cscw_windows");
  timing_end("cscw_windows", s);
  if (msrep_status st = scan::device_scan<int32_t, scan::SumOp>(inv_cnt, inv_off, W.nwin + 1,
                                                                inv_agg, false, s))
    return st;
  const int64_t pairs = static_cast<int64_t>(W.P) * kWinMax;
  hipLaunchKernelGGL(cscw_inv_fill, dim3(static_cast<unsigned>((pairs + 255) / 256)), dim3(256), 0,
                     s, wlist, wcnt, W.P, inv_off, inv_cnt, inv_list);
  MSREP_LAUNCHED("cscw_inv_fill");
  return MSREP_OK;
}

template <int VT>
msrep_status cscw_numeric(const msrep_mat *A, const msrep_part *parts, const int32_t *lptr,
                          int32_t np, const void *x, void *y, double alpha, double beta,
                          const CscLayout &L, const CscwLayout &W, char *b, hipStream_t s) {
  using Tr = vt_traits<VT>;
  using T = typename Tr::T;
  const int32_t *wlist = reinterpret_cast<const int32_t *>(b + W.wlist);
  const int32_t *wcnt = reinterpret_cast<const int32_t *>(b + W.wcnt);
  const int32_t *flags = reinterpret_cast<const int32_t *>(b + W.flags);
  const int32_t *inv_off = reinterpret_cast<const int32_t *>(b + W.inv_off);
  const int32_t *inv_list = reinterpret_cast<const int32_t *>(b + W.inv_list);
  double *part = reinterpret_cast<double *>(b + L.prod + W.part);
  double *yacc = reinterpret_cast<double *>(b + L.prod + W.yacc);
  {
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      return fail(MSREP_ERR_HIP, "msrep_spmv: cannot query the LDS size");
    if (static_cast<size_t>(lds) < cscw_lds<4>())
      return fail(MSREP_ERR_UNSUPPORTED, "msrep_spmv: row windows need %zu bytes of LDS per block "
                  "(the device offers %d)", cscw_lds<4>(), lds);
  }
  hipLaunchKernelGGL(cscw_zero, dim3(static_cast<unsigned>(std::min<int64_t>((A->m + 255) / 256, 8192))),
                     dim3(256), 0, s, flags, yacc, static_cast<int64_t>(A->m));
  MSREP_LAUNCHED("cscw_zero");
  timing_begin("cscw_tile", s);
  if (A->fmt == MSREP_CSC)
    hipLaunchKernelGGL((cscw_tile<VT, 4, false>), dim3(W.P), dim3(kWinWaves * kWave), cscw_lds<4>(),
                       s, A->idx, A->idx2, static_cast<const typename Tr::V *>(A->val), parts, lptr,
                       np, W.P, static_cast<const T *>(x), A->m, A->n, wlist, wcnt, part, yacc);
  else
    hipLaunchKernelGGL((cscw_tile<VT, 4, true>), dim3(W.P), dim3(kWinWaves * kWave), cscw_lds<4>(),
                       s, A->idx, A->idx2, static_cast<const typename Tr::V *>(A->val), parts, lptr,
                       np, W.P, static_cast<const T *>(x), A->m, A->n, wlist, wcnt, part, yacc);
  MSREP_LAUNCHED("cscw_tile");
  timing_end("cscw_tile", s);
  timing_begin("cscw_merge", s);
  if (beta == 0.0)
    hipLaunchKernelGGL((cscw_merge<T, true>), dim3(static_cast<unsigned>(W.nwin)), dim3(kWinMergeBlock),
                       0, s, inv_off, inv_list, flags, part, yacc, A->m, static_cast<T *>(y), alpha,
                       beta);
  else
    hipLaunchKernelGGL((cscw_merge<T, false>), dim3(static_cast<unsigned>(W.nwin)), dim3(kWinMergeBlock),
                       0, s, inv_off, inv_list, flags, part, yacc, A->m, static_cast<T *>(y), alpha,
                       beta);
  MSREP_LAUNCHED("cscw_merge");
  timing_end("cscw_merge", s);
  return MSREP_OK;
}

// CSC, COO_COL, COO_ANY.  pf == 3: the windowed path; otherwise the bucketed
// path with product layout pf.  The structure phase (msrep_spmv_prepare,
// which has no tune) builds the structure of both paths.  Matrices with more
// rows than the buckets cover (2^26) take the windowed path whatever pf is:
// its spill vector takes any row, so it has no row limit.
template <int VT>
msrep_status launch_csc_any(const msrep_mat *A, const msrep_part *parts, const int32_t *lptr,
                            int32_t np, const void *x, void *y, double alpha, double beta, int K,
                            int wpb, int pf, void *ws, int phase, hipStream_t s) {
  using Acc = typename vt_traits<VT>::A;
  CscLayout L;
  const bool bucketed_ok = csc_layout(A->m, A->nnz, np, sizeof(Acc), L);
  if (!bucketed_ok) L = CscLayout{};  // windowed only: its regions from the workspace's start
  if (pf == 3 || phase == kPhaseStructure || !bucketed_ok) {
    CscwLayout W;
    cscw_place(A, np, L, W);
    char *b = static_cast<char *>(ws);
    if (phase != kPhaseNumeric)
      if (msrep_status st = cscw_structure(A, parts, np, W, b, s)) return st;
    if (phase == kPhaseStructure) {
      if (!bucketed_ok) return MSREP_OK;
      // and the bucketed path's structure, for calls with either layout
      return K == 8 ? launch_csc<VT, 8, false>(A, parts, lptr, np, x, y, alpha, beta, wpb, ws, phase, s)
                    : launch_csc<VT, 4, false>(A, parts, lptr, np, x, y, alpha, beta, wpb, ws, phase, s);
    }
    return cscw_numeric<VT>(A, parts, lptr, np, x, y, alpha, beta, L, W, b, s);
  }
  if (pf == 1)
    return K == 8 ? launch_csc<VT, 8, true>(A, parts, lptr, np, x, y, alpha, beta, wpb, ws, phase, s)
                  : launch_csc<VT, 4, true>(A, parts, lptr, np, x, y, alpha, beta, wpb, ws, phase, s);
  return K == 8 ? launch_csc<VT, 8, false>(A, parts, lptr, np, x, y, alpha, beta, wpb, ws, phase, s)
                : launch_csc<VT, 4, false>(A, parts, lptr, np, x, y, alpha, beta, wpb, ws, phase, s);
}

template <int VT, int K, bool B0>
msrep_status dispatch_rows(const msrep_mat *A, const msrep_part *parts, const int32_t *lptr,
                           int32_t np, const void *x, void *y, double alpha, double beta,
                           int wpb, int pf, int resident, double *carry, hipStream_t s) {
  if (A->fmt == MSREP_CSR)
    return launch_csr<VT, K, B0>(A, parts, lptr, np, x, y, alpha, beta, wpb, pf, resident, carry,
                                 s);
  return launch_coo<VT, K, B0>(A, parts, np, x, y, alpha, beta, wpb, resident, carry, s);
}

template <int VT>
msrep_status dispatch_vt(const msrep_mat *A, const msrep_part *parts, const int32_t *lptr,
                         int32_t np, const void *x, void *y, double alpha, double beta, int K,
                         int wpb, int pf, int resident, double *carry, int phase, hipStream_t s) {
  using T = typename vt_traits<VT>::T;
  const bool b0 = beta == 0.0;
  msrep_status st;
  if (bucketed_fmt(A->fmt))  // carry is the whole workspace here
    return launch_csc_any<VT>(A, parts, lptr, np, x, y, alpha, beta, K, wpb, pf, carry, phase, s);
  if (phase == kPhaseStructure) return MSREP_OK;  // CSR, COO: no structure-only work
  if (K == 8)
    st = b0 ? dispatch_rows<VT, 8, true>(A, parts, lptr, np, x, y, alpha, beta, wpb, pf, resident, carry, s)
            : dispatch_rows<VT, 8, false>(A, parts, lptr, np, x, y, alpha, beta, wpb, pf, resident, carry, s);
  else
    st = b0 ? dispatch_rows<VT, 4, true>(A, parts, lptr, np, x, y, alpha, beta, wpb, pf, resident, carry, s)
            : dispatch_rows<VT, 4, false>(A, parts, lptr, np, x, y, alpha, beta, wpb, pf, resident, carry, s);
  if (st) return st;
  if (np > 1) return launch_merge_rows(A, parts, np, carry, y, alpha, beta, 1, 0, 1, s);
  return MSREP_OK;
}

}  // namespace

msrep_status launch_merge_rows(const msrep_mat *A, const msrep_part *parts, int32_t np,
                               const double *carry, void *y, double alpha, double beta,
                               int64_t ldy, int64_t cstride, int ncols, hipStream_t s) {
  const int g = (np + kMergeBlock - 1) / kMergeBlock;
  const bool b0 = beta == 0.0;
  timing_begin("merge_rows", s);
  if (A->vtype == MSREP_F64) {
    if (b0)
      hipLaunchKernelGGL((merge_rows<double, true>), dim3(g, ncols), dim3(kMergeBlock), 0, s,
                         parts, np, carry, static_cast<double *>(y), A->m, alpha, beta, ldy, cstride);
    else
      hipLaunchKernelGGL((merge_rows<double, false>), dim3(g, ncols), dim3(kMergeBlock), 0, s,
                         parts, np, carry, static_cast<double *>(y), A->m, alpha, beta, ldy, cstride);
  } else {
    if (b0)
      hipLaunchKernelGGL((merge_rows<float, true>), dim3(g, ncols), dim3(kMergeBlock), 0, s,
                         parts, np, carry, static_cast<float *>(y), A->m, alpha, beta, ldy, cstride);
    else
      hipLaunchKernelGGL((merge_rows<float, false>), dim3(g, ncols), dim3(kMergeBlock), 0, s,
                         parts, np, carry, static_cast<float *>(y), A->m, alpha, beta, ldy, cstride);
  }
  MSREP_LAUNCHED("merge_rows");
  timing_end("merge_rows", s);
  return MSREP_OK;
}

msrep_status resolve_tune(const msrep_tune *tune, int *K, int *wpb, int *pf, int *resident,
                          const char *who) {
  *K = 4;
  *wpb = 4;
  *pf = 2;
  *resident = 0;
  if (!tune) return MSREP_OK;
  if (tune->pipeline < 0 || tune->pipeline > 3)
    return fail(MSREP_ERR_ARG, "%s: pipeline must be 0..3 (got %d)", who, tune->pipeline);
  if (tune->pipeline) *pf = tune->pipeline;
  if (tune->k_per_lane != 0 && tune->k_per_lane != 4 && tune->k_per_lane != 8)
    return fail(MSREP_ERR_ARG, "%s: k_per_lane must be 4 or 8 (got %d)", who, tune->k_per_lane);
  if (tune->waves_per_wg < 0 || tune->waves_per_wg > 8)
    return fail(MSREP_ERR_ARG, "%s: waves_per_wg must be 1..8 (got %d)", who, tune->waves_per_wg);
  if (tune->resident != 0 && tune->resident != 1)
    return fail(MSREP_ERR_ARG, "%s: resident must be 0 or 1 (got %d)", who, tune->resident);
  if (tune->k_per_lane) *K = tune->k_per_lane;
  if (tune->waves_per_wg) *wpb = tune->waves_per_wg;
  *resident = tune->resident;
  return MSREP_OK;
}

msrep_status spmv_launch_phase(const msrep_mat *A, const msrep_part *parts, const int32_t *lptr,
                               int32_t np, const void *x, void *y, double alpha, double beta,
                               int K, int wpb, int pf, int resident, double *carry, int phase,
                               hipStream_t s) {
  switch (A->vtype) {
    case MSREP_F64:
      return dispatch_vt<MSREP_F64>(A, parts, lptr, np, x, y, alpha, beta, K, wpb, pf, resident, carry, phase, s);
    case MSREP_F32:
      return dispatch_vt<MSREP_F32>(A, parts, lptr, np, x, y, alpha, beta, K, wpb, pf, resident, carry, phase, s);
    default:
      return dispatch_vt<MSREP_BF16>(A, parts, lptr, np, x, y, alpha, beta, K, wpb, pf, resident, carry, phase, s);
  }
}

msrep_status spmv_launch(const msrep_mat *A, const msrep_part *parts, const int32_t *lptr,
                         int32_t np, const void *x, void *y, double alpha, double beta, int K,
                         int wpb, int pf, int resident, double *carry, hipStream_t s) {
  return spmv_launch_phase(A, parts, lptr, np, x, y, alpha, beta, K, wpb, pf, resident, carry,
                           kPhaseAll, s);
}

}  // namespace msrep

using namespace msrep;

extern "C" const char *msrep_last_error(void) { return last_error().c_str(); }

extern "C" int32_t msrep_vtype_bytes(int32_t vtype) { return value_bytes(vtype); }

namespace msrep {


size_t spmv_ws_bytes(int32_t fmt, int32_t vtype, int32_t m, int64_t nnz, int32_t np) {
  if (bucketed_fmt(fmt)) {
    CscLayout L;
    const int pb = vtype == MSREP_F64 ? 8 : 4;
    if (!csc_layout(m, nnz, np, pb, L)) L = CscLayout{};  // windowed only (over 2^26 rows)
    // the windowed path's numeric regions overlap the bucketed ones, its
    // structure follows both
    CscwLayout W;
    cscw_layout(m, nnz, np, L, W);
    return W.struct_end;
  }
  return align_up(16 * static_cast<size_t>(np), 256);
}

}  // namespace msrep

extern "C" size_t msrep_spmv_ws_bytes(const msrep_mat *A, int32_t np) {
  if (!A || np <= 0 || A->m < 0 || A->nnz < 0) return 0;
  return spmv_ws_bytes(A->fmt, A->vtype, A->m, A->nnz, np);
}

namespace {

// msrep_spmv and its prepare / prepared split: the same checks, then the
// kernels of `phase`.
msrep_status spmv_entry(const msrep_mat *A, const msrep_part *parts_d, const int32_t *lptr_d,
                        int32_t np, const void *x_d, void *y_d, double alpha, double beta,
                        const msrep_tune *tune, void *ws_d, size_t ws_bytes, void *stream,
                        int phase, const char *who) {
  if (msrep_status st = check_mat(A, who)) return st;
  if (np <= 0) return fail(MSREP_ERR_ARG, "%s: np must be positive (got %d)", who, np);
  if (!parts_d) return fail(MSREP_ERR_ARG, "%s: parts_d is NULL", who);
  if ((A->fmt == MSREP_CSR || A->fmt == MSREP_CSC) && !lptr_d)
    return fail(MSREP_ERR_ARG, "%s: lptr_d is NULL", who);
  if (phase != kPhaseStructure) {
    if (A->m > 0 && !y_d) return fail(MSREP_ERR_ARG, "%s: y_d is NULL", who);
    if (A->nnz > 0 && !x_d) return fail(MSREP_ERR_ARG, "%s: x_d is NULL", who);
  }
  int K, wpb, pf, resident;
  if (msrep_status st = resolve_tune(tune, &K, &wpb, &pf, &resident, who)) return st;
  if (pf == 3 && !bucketed_fmt(A->fmt))
    return fail(MSREP_ERR_ARG, "%s: pipeline 3 (row windows) is a CSC / column-merge layout", who);
  // x, y and the local pointers are addressed through 32-bit buffer offsets
  const uint64_t xb = static_cast<uint64_t>(A->n) * vec_bytes(A->vtype);
  const uint64_t yb = static_cast<uint64_t>(A->m) * vec_bytes(A->vtype);
  if (xb >= (uint64_t(1) << 32) || yb >= (uint64_t(1) << 32) ||
      (static_cast<uint64_t>(major_dim(A)) + 1) * 4 >= (uint64_t(1) << 32))
    return fail(MSREP_ERR_UNSUPPORTED, "%s: x or y larger than 4 GiB", who);
  const size_t need = msrep_spmv_ws_bytes(A, np);
  if (!ws_d || ws_bytes < need)
    return fail(MSREP_ERR_SIZE, "%s: workspace of %zu bytes needed (got %zu)", who, need,
                ws_d ? ws_bytes : size_t(0));
  if (A->m == 0) return ok();
  if (msrep_status st = spmv_launch_phase(A, parts_d, lptr_d, np, x_d, y_d, alpha, beta, K, wpb,
                                          pf, resident, static_cast<double *>(ws_d), phase,
                                          as_stream(stream)))
    return st;
  return ok();
}

}  // namespace

extern "C" msrep_status msrep_spmv(const msrep_mat *A, const msrep_part *parts_d,
                                   const int32_t *lptr_d, int32_t np, const void *x_d, void *y_d,
                                   double alpha, double beta, const msrep_tune *tune, void *ws_d,
                                   size_t ws_bytes, void *stream) {
  return spmv_entry(A, parts_d, lptr_d, np, x_d, y_d, alpha, beta, tune, ws_d, ws_bytes, stream,
                    kPhaseAll, "msrep_spmv");
}

extern "C" msrep_status msrep_spmv_prepare(const msrep_mat *A, const msrep_part *parts_d,
                                           const int32_t *lptr_d, int32_t np, void *ws_d,
                                           size_t ws_bytes, void *stream) {
  return spmv_entry(A, parts_d, lptr_d, np, nullptr, nullptr, 1.0, 0.0, nullptr, ws_d, ws_bytes,
                    stream, kPhaseStructure, "msrep_spmv_prepare");
}

extern "C" msrep_status msrep_spmv_prepared(const msrep_mat *A, const msrep_part *parts_d,
                                            const int32_t *lptr_d, int32_t np, const void *x_d,
                                            void *y_d, double alpha, double beta,
                                            const msrep_tune *tune, void *ws_d, size_t ws_bytes,
                                            void *stream) {
  return spmv_entry(A, parts_d, lptr_d, np, x_d, y_d, alpha, beta, tune, ws_d, ws_bytes, stream,
                    kPhaseNumeric, "msrep_spmv_prepared");
}

// ------------------------------------------------ no-allocation variant
// The boundary-merge carries of msrep_spmv (two FP64 slots per partition)
// taken from a file-scope device array instead of a caller workspace, for
// callers that cannot allocate.  In host code `scratch` names a host-side
// stand-in; its device address comes from hipGetSymbolAddress, once per
// device, and only that address is ever passed to a kernel.
namespace {

constexpr int32_t kNoAllocMaxParts = 1 << 19;  // 8 MiB of carries per device
__device__ __align__(256) double scratch[2 * static_cast<size_t>(kNoAllocMaxParts)];

std::mutex scratch_mu;
std::map<int, double *> scratch_addr;  // device ordinal -> address of its copy

// The calling thread's current device's copy of `scratch`.
msrep_status scratch_on_current_device(double **out, const char *who) {
  int dev = 0;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess)
    return fail(MSREP_ERR_HIP, "%s: hipGetDevice failed: %s", who, hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(scratch_mu);
  auto it = scratch_addr.find(dev);
  if (it == scratch_addr.end()) {
    void *p = nullptr;
    const hipError_t g = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (g != hipSuccess || !p)
      return fail(MSREP_ERR_HIP, "%s: hipGetSymbolAddress(scratch) failed on device %d: %s", who,
                  dev, hipGetErrorString(g));
    it = scratch_addr.emplace(dev, static_cast<double *>(p)).first;
  }
  *out = it->second;
  return MSREP_OK;
}

}  // namespace

extern "C" int32_t msrep_spmv_noalloc_max_parts(void) { return kNoAllocMaxParts; }

extern "C" msrep_status msrep_spmv_noalloc(const msrep_mat *A, const msrep_part *parts_d,
                                           const int32_t *lptr_d, int32_t np, const void *x_d,
                                           void *y_d, double alpha, double beta,
                                           const msrep_tune *tune, void *stream) {
  const char *who = "msrep_spmv_noalloc";
  if (msrep_status st = check_mat(A, who)) return st;
  if (A->fmt != MSREP_CSR && A->fmt != MSREP_COO)
    return fail(MSREP_ERR_UNSUPPORTED, "%s: CSR and row-sorted COO only (format %d)", who,
                A->fmt);
  if (np <= 0) return fail(MSREP_ERR_ARG, "%s: np must be positive (got %d)", who, np);
  if (np > kNoAllocMaxParts)
    return fail(MSREP_ERR_SIZE, "%s: np=%d exceeds the %d partitions of the static scratch", who,
                np, kNoAllocMaxParts);
  double *carry = nullptr;
  if (msrep_status st = scratch_on_current_device(&carry, who)) return st;
  // the same checks and kernels as msrep_spmv, on the scratch's carries
  return spmv_entry(A, parts_d, lptr_d, np, x_d, y_d, alpha, beta, tune, carry,
                    2 * sizeof(double) * static_cast<size_t>(kNoAllocMaxParts), stream,
                    kPhaseAll, who);
}
