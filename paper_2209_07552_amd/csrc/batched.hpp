// Descriptors and kernels shared by the batched plan and the server: one
// persistent launch drains a list of (matrix, partition) work items, each
// processed by the CSR wave routine, and one launch merges the rows split
// between partitions of every matrix.
#pragma once

#include "spmv_csr.hpp"

namespace msrep {

struct BatchMat {
  const int32_t *col;
  const void *val;
  const msrep_part *parts;
  const int32_t *lptr;
  int32_t m, n, np, _pad;
  double *carry;  // two FP64 slots per partition of this matrix
};
struct BatchXY {
  const void *x;
  void *y;
};

// wave_begin[w] .. wave_begin[w+1]-1 are the work items of wavefront w.
template <int VT, int K, bool BETA0>
__global__ __launch_bounds__(512) void spmv_batched_persistent(
    const BatchMat *__restrict__ mats, const BatchXY *__restrict__ xy,
    const int2 *__restrict__ items, const int64_t *__restrict__ wave_begin, int32_t n_waves,
    double alpha, double beta) {
  using Tr = vt_traits<VT>;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int wid = threadIdx.x / kWave;
  const int wpb = blockDim.x / kWave;
  const int w = xcd_block(blockIdx.x, gridDim.x) * wpb + wid;
  if (w >= n_waves) return;
  unsigned char *my = lds_raw + wid * seg_lds_per_wave<VT, K>();
  const int64_t lo = uniform(wave_begin[w]), hi = uniform(wave_begin[w + 1]);
  for (int64_t it = lo; it < hi; ++it) {
    const int2 wk = items[it];
    const int32_t k = uniform(wk.x), p = uniform(wk.y);
    const BatchMat *M = mats + k;
    const int32_t *col = uniform(M->col);
    const typename Tr::V *val = static_cast<const typename Tr::V *>(uniform(M->val));
    const msrep_part *parts = uniform(M->parts);
    const int32_t *lptr = uniform(M->lptr);
    const int32_t m = uniform(M->m), n = uniform(M->n), np = uniform(M->np);
    double *carry = uniform(M->carry);
    const typename Tr::T *x = static_cast<const typename Tr::T *>(uniform(xy[k].x));
    typename Tr::T *y = static_cast<typename Tr::T *>(uniform(xy[k].y));
    csr_partition<VT, K, BETA0>(col, val, parts, lptr, np, p, x, y, m, n, alpha, beta, carry, my);
    wave_lds_sync();
  }
}

// Boundary merge of every matrix: one thread per work item (see merge_rows).
template <typename T, bool BETA0>
__global__ __launch_bounds__(256) void merge_batched(const BatchMat *__restrict__ mats,
                                                     const BatchXY *__restrict__ xy,
                                                     const int2 *__restrict__ items,
                                                     int64_t n_items, double alpha, double beta) {
  const int64_t it = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (it >= n_items) return;
  const int2 wk = items[it];
  const BatchMat M = mats[wk.x];
  const int32_t p = wk.y;
  const msrep_part P = M.parts[p];
  if (P.end_idx < P.start_idx || !P.end_flag) return;
  if (P.start_flag && P.start_row == P.end_row) return;
  const int32_t r = P.end_row;
  const double tot = split_row_total(M.parts, M.np, M.carry, p, r);
  if (r < 0 || r >= M.m) return;
  T *y = static_cast<T *>(xy[wk.x].y);
  y[r] = static_cast<T>(BETA0 ? alpha * tot : alpha * tot + beta * static_cast<double>(y[r]));
}

// Contiguous runs of work items with about equal cost, one per wavefront:
// begin has n_waves + 1 entries.
inline void equal_work_runs(const int64_t *cost, int64_t n_items, int32_t n_waves, int64_t *begin) {
  int64_t total = 0;
  for (int64_t i = 0; i < n_items; ++i) total += cost[i];
  int64_t acc = 0, it = 0;
  begin[0] = 0;
  for (int32_t w = 1; w < n_waves; ++w) {
    const int64_t target = (total * w) / n_waves;
    while (it < n_items && acc + cost[it] <= target) acc += cost[it++];
    begin[w] = it;
  }
  begin[n_waves] = n_items;
}

// Cost of partition p of an np-way split of a matrix (its nonzeros plus its
// share of rows, whose y each wavefront writes).
inline int64_t item_cost(int64_t nnz, int32_t m, int32_t np, int32_t p) {
  const int64_t nz = (static_cast<int64_t>(p + 1) * nnz) / np - (static_cast<int64_t>(p) * nnz) / np;
  return nz + (static_cast<int64_t>(m) + np - 1) / np;
}

}  // namespace msrep
