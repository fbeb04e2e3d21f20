// msrep_autotune: choose the partition size (nonzeros per wavefront, i.e. the
// np of the equal-nnz split) and the launch shape (nonzeros per lane per
// chunk, wavefronts per workgroup, CSR pipeline depth, resident grid) for one
// matrix by timing every candidate on the device: build the partitions, run
// the SpMV a few times, keep the fastest median.  Synchronises the stream.
#include <algorithm>
#include <vector>

#include "common.hpp"

namespace msrep {
msrep_status spmv_launch(const msrep_mat *A, const msrep_part *parts, const int32_t *lptr,
                         int32_t np, const void *x, void *y, double alpha, double beta, int K,
                         int wpb, int pf, int resident, double *carry, hipStream_t s);
size_t spmv_ws_bytes(int32_t fmt, int32_t vtype, int32_t m, int64_t nnz, int32_t np);
namespace {

constexpr int kNpw[] = {256, 512, 1024, 2048, 4096};
constexpr int kK[] = {4, 8};
constexpr int kWpb[] = {2, 4, 8};
constexpr int kPf[] = {1, 2, 3};  // CSR load depth; column merge: layouts, 3 = row windows
constexpr int kResident[] = {0, 1};
constexpr int kReps = 3;

struct TuneWs {
  size_t parts, lptr, y, carry, total;
  int32_t np_max;
};

TuneWs tune_ws(const msrep_mat *A) {
  TuneWs w{};
  const int64_t npm = std::max<int64_t>(1, (A->nnz + kNpw[0] - 1) / kNpw[0]);
  w.np_max = static_cast<int32_t>(std::min<int64_t>(npm, INT32_MAX / 4));
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o += align_up(b ? b : 1, 256);
    return at;
  };
  w.parts = take(sizeof(msrep_part) * w.np_max);
  w.lptr = take(4 * static_cast<size_t>(msrep_lptr_bound(major_dim(A), w.np_max)));
  w.y = take(static_cast<size_t>(vec_bytes(A->vtype)) * A->m);
  // the SpMV workspace (merge slots, or the CSC buckets) at the largest np
  w.carry = take(spmv_ws_bytes(A->fmt, A->vtype, A->m, A->nnz, w.np_max));
  w.total = o;
  return w;
}

}  // namespace
}  // namespace msrep

using namespace msrep;

extern "C" size_t msrep_autotune_ws_bytes(const msrep_mat *A) {
  if (!A || A->nnz < 0 || A->m < 0 || A->n < 0) return 0;
  return tune_ws(A).total;
}

extern "C" msrep_status msrep_autotune(const msrep_mat *A, const void *x_d, void *ws_d,
                                       size_t ws_bytes, msrep_tune *out, void *stream) {
  if (msrep_status st = check_mat(A, "msrep_autotune")) return st;
  if (!out) return fail(MSREP_ERR_ARG, "msrep_autotune: out is NULL");
  if (A->nnz > 0 && !x_d) return fail(MSREP_ERR_ARG, "msrep_autotune: x_d is NULL");
  const TuneWs w = tune_ws(A);
  if (!ws_d || ws_bytes < w.total)
    return fail(MSREP_ERR_SIZE, "msrep_autotune: workspace of %zu bytes needed (got %zu)", w.total,
                ws_d ? ws_bytes : size_t(0));
  hipStream_t s = as_stream(stream);
  char *b = static_cast<char *>(ws_d);
  msrep_part *parts = reinterpret_cast<msrep_part *>(b + w.parts);
  int32_t *lptr = reinterpret_cast<int32_t *>(b + w.lptr);
  void *y = b + w.y;
  double *carry = reinterpret_cast<double *>(b + w.carry);
  hipEvent_t e0, e1;
  MSREP_HIP(hipEventCreate(&e0));
  MSREP_HIP(hipEventCreate(&e1));
  msrep_tune best{4, 4, 0, 1024, 2, 0};
  float best_ms = 1e30f;
  msrep_status err = MSREP_OK;
  for (int npw : kNpw) {
    if (err) break;
    const int64_t np64 = std::max<int64_t>(1, (A->nnz + npw - 1) / npw);
    if (np64 > w.np_max) continue;
    const int32_t np = static_cast<int32_t>(np64);
    if ((err = msrep_build_partition(A, np, parts, lptr, msrep_lptr_bound(major_dim(A), np),
                                     nullptr, stream)))
      break;
    for (int K : kK)
      for (int wpb : kWpb)
        for (int pf : kPf)
          for (int res : kResident) {
            if (err) break;
            // CSC has neither choice (its producer shapes are fixed)
            const bool bucketed = bucketed_fmt(A->fmt);
            if (bucketed && (res == 1 || wpb != kWpb[0])) continue;
            if (A->fmt == MSREP_COO && pf == 1) continue;  // CSR pipelines, CSC layouts
            if (pf == 3 && !bucketed) continue;            // row windows: column merge only
            if ((err = spmv_launch(A, parts, lptr, np, x_d, y, 1.0, 0.0, K, wpb, pf, res, carry, s)))
              break;
            std::vector<float> t;
            for (int r = 0; r < kReps && !err; ++r) {
              if (hipEventRecord(e0, s) != hipSuccess) err = fail(MSREP_ERR_HIP, "hipEventRecord");
              if (!err)
                err = spmv_launch(A, parts, lptr, np, x_d, y, 1.0, 0.0, K, wpb, pf, res, carry, s);
              if (!err && hipEventRecord(e1, s) != hipSuccess)
                err = fail(MSREP_ERR_HIP, "hipEventRecord");
              float ms = 0.f;
              if (!err && (hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                err = fail(MSREP_ERR_HIP, "timing failed");
              t.push_back(ms);
            }
            if (err) break;
            std::sort(t.begin(), t.end());
            const float med = t[t.size() / 2];
            if (med < best_ms) {
              best_ms = med;
              best = msrep_tune{K, wpb, res, npw, pf, 0};
            }
          }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err) return err;
  *out = best;
  return ok();
}
