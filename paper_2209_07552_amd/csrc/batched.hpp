// Descriptors and kernels shared by the batched plan and the server: one
// persistent launch drains a list of (matrix, partition) work items, each
// processed by the CSR wave routine, and one launch merges the rows split
// between partitions of every matrix.
//
// Both callers describe their work items through a source type with
//   __device__ void get(int64_t it, BItem &out) const;   // item it (it may
//                                                        // differ per lane)
//   __device__ void group(int32_t g, int32_t G, int64_t &lo, int64_t &hi) const;
//                                  // items [lo, hi) of group g of G
//   int64_t n_items; int32_t n_waves;
// The items are split into one contiguous group per XCD; the wavefronts of
// an XCD sweep its group together (wavefront j of the XCD's W takes items
// lo + j, lo + j + W, ...), so at any moment an XCD works on a window of
// consecutive items, i.e. on a few matrices, whose x vectors its L2 holds.
// The batched plan reads a precomputed item list from device memory; a
// serving tick (serve.hip) passes its active requests in the kernel
// arguments, so a tick needs no table copy from the host.
#pragma once

#include "spmm_csr.hpp"

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

// One work item resolved: partition p of a matrix and its vectors.
struct BItem {
  const int32_t *col;
  const void *val;
  const msrep_part *parts;
  const int32_t *lptr;
  double *carry;
  const void *x;
  void *y;
  int32_t m, n, np, p;
  int64_t ldy;  // y's row stride in elements (1: a vector; k: a column of an m x k block)
};

__device__ __forceinline__ void bitem_from(const BatchMat &M, const BatchXY &xy, int32_t p,
                                           BItem &o) {
  o.col = M.col;
  o.val = M.val;
  o.parts = M.parts;
  o.lptr = M.lptr;
  o.carry = M.carry;
  o.x = xy.x;
  o.y = xy.y;
  o.m = M.m;
  o.n = M.n;
  o.np = M.np;
  o.p = p;
  o.ldy = 1;
}

// The batched plan's items: a device list of (matrix, partition) pairs and
// its split into equal-work groups, one per XCD.
struct PlanSrc {
  const BatchMat *mats;
  const BatchXY *xy;
  const int2 *items;
  const int64_t *group_begin;  // G + 1 entries, G = min(8, grid)
  int64_t n_items;
  int32_t n_waves, _pad;
  __device__ void get(int64_t it, BItem &o) const {
    const int2 wk = items[it];
    bitem_from(mats[wk.x], xy[wk.x], wk.y, o);
  }
  __device__ void group(int32_t g, int32_t, int64_t &lo, int64_t &hi) const {
    lo = uniform(group_begin[g]);
    hi = uniform(group_begin[g + 1]);
  }
};

// Resident wavefronts; those of one XCD (blocks are dealt to the XCDs round
// robin by id) sweep that XCD's group of items together.
template <int VT, int K, bool BETA0, int PF, class Src>
__global__ __launch_bounds__(512) void spmv_items_persistent(const Src src, double alpha,
                                                            double beta) {
  using Tr = vt_traits<VT>;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int wid = threadIdx.x / kWave;
  const int wpb = blockDim.x / kWave;
  const int nb = static_cast<int>(gridDim.x);
  const int G = nb < kXcds ? nb : kXcds;
  const int g = static_cast<int>(blockIdx.x) % G;
  const int j = (static_cast<int>(blockIdx.x) / G) * wpb + wid;  // wavefront within the group
  const int wg = (nb / G + (g < nb % G ? 1 : 0)) * wpb;             // wavefronts of the group
  unsigned char *my = lds_raw + wid * seg_lds_per_wave<VT, K>();
  int64_t lo, hi;
  src.group(g, G, lo, hi);
  for (int64_t it = lo + j; it < hi; it += wg) {
    BItem b;
    src.get(it, b);
    const int32_t m = uniform(b.m), n = uniform(b.n), np = uniform(b.np), p = uniform(b.p);
    csr_partition<VT, K, BETA0, PF>(
        uniform(b.col), static_cast<const typename Tr::V *>(uniform(b.val)), uniform(b.parts),
        uniform(b.lptr), np, p, static_cast<const typename Tr::T *>(uniform(b.x)),
        static_cast<typename Tr::T *>(uniform(b.y)), m, n, alpha, beta, uniform(b.carry), my);
    wave_lds_sync();
  }
}

// Boundary merge of every matrix at once: the segmented sum of merge_rows
// (spmv_csr.hpp) run over the concatenated work items.  Chains never cross
// matrices, since the first partition of a matrix has no start flag and so
// starts a segment.  The thread of the item where a split row ends writes
// that row of its matrix's y.
template <class Src>
__device__ __forceinline__ MSeg item_seg(const Src &src, int64_t q, BItem &b, MPart &P) {
  src.get(q, b);
  P = mpart_load(b.parts, b.p);
  return mpart_seg(P, b.carry[2 * static_cast<int64_t>(b.p)],
                   b.carry[2 * static_cast<int64_t>(b.p) + 1]);
}

template <typename T, bool BETA0, class Src>
__global__ __launch_bounds__(kMergeBlock) void merge_items(const Src src, double alpha,
                                                           double beta) {
  __shared__ double sh_s[kMergeWaves], sh_c[kMergeWaves];
  __shared__ int sh_f[kMergeWaves];
  const int t = threadIdx.x;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kMergeBlock;
  const int64_t q = base + t;
  MPart P{0, -1, 0, 0};
  BItem b{};
  MSeg own{0.0, 0.0, 0};
  double hd = 0.0;
  if (q < src.n_items) {
    own = item_seg(src, q, b, P);
    hd = b.carry[2 * static_cast<int64_t>(b.p)];
  }
  // the 64 items just before the block, loaded up front by wave 0
  const int64_t near = base > kWave ? base - kWave : 0;
  MSeg look{0.0, 0.0, 0};
  if (t < kWave && near + t < base) {
    BItem bb;
    MPart PP;
    look = item_seg(src, near + t, bb, PP);
  }
  MSeg excl;
  (void)block_mseg_scan(own, excl, sh_s, sh_c, sh_f);
  const bool last = P.er >= P.sr && P.sf && !(P.ef && P.sr == P.er);  // a split row ends here
  MSeg at = mseg_cat(excl, MSeg{hd, 0.0, 0});
  const bool need = last && !at.f;  // the row began before this block
  if (__syncthreads_or(need)) {
    if (t < kWave) {
      wave_mseg_scan(look);
      if (t == kWave - 1) {
        sh_s[0] = look.s;
        sh_c[0] = look.c;
        sh_f[0] = look.f;
      }
    }
    __syncthreads();
    MSeg acc{sh_s[0], sh_c[0], sh_f[0]};
    __syncthreads();
    constexpr int64_t kSpan = kMergeBlock * kMergeLook;
    int64_t hi = near;
    while (hi > 0 && !acc.f) {
      const int64_t lo = hi > kSpan ? hi - kSpan : 0;
      MSeg w{0.0, 0.0, 0};
#pragma unroll
      for (int j = 0; j < kMergeLook; ++j) {
        const int64_t qq = lo + t * kMergeLook + j;
        if (qq < hi) {
          BItem bb;
          MPart PP;
          w = mseg_cat(w, item_seg(src, qq, bb, PP));
        }
      }
      MSeg wex;
      acc = mseg_cat(block_mseg_scan(w, wex, sh_s, sh_c, sh_f), acc);
      hi = lo;
    }
    if (need) at = mseg_cat(acc, at);
  }
  if (!last) return;
  const int32_t r = P.sr;
  if (r < 0 || r >= b.m) return;
  const double tot = at.s + at.c;
  T *yr = static_cast<T *>(b.y) + static_cast<int64_t>(r) * b.ldy;
  *yr = static_cast<T>(BETA0 ? alpha * tot : alpha * tot + beta * static_cast<double>(*yr));
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
