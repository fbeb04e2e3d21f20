// Equal-nnz partition build for pCSR / pCSC / pCOO (msRep Sec. 3.2,
// Algorithms 2, 4 and 6), entirely on the GPU: one thread per partition finds
// the start/end rows by bisection (O(np log m)), then the local pointers are
// written by a second kernel (O(m)), the offload the paper's optimised variant
// applies (Sec. 4.1).  Every partition depends on nothing but A and its own
// index, so both kernels are embarrassingly parallel.  The paper's Baseline
// split (equal rows or columns per partition, Sec. 5.3) is built the same way
// into the same records, for comparison runs.
#include "common.hpp"

namespace msrep {
namespace {

// Row containing nonzero k: the largest r in [0, rows) with ptr[r] <= k.
// Requires 0 <= k < ptr[rows] for a meaningful answer; always returns a value
// in [0, rows) (rows >= 1) and never reads outside ptr[0..rows].
__device__ int32_t row_containing(const int32_t *__restrict__ ptr, int32_t rows, int64_t k) {
  int32_t lo = 0, hi = rows;
  while (hi - lo > 1) {
    const int32_t mid = lo + ((hi - lo) >> 1);
    if (static_cast<int64_t>(ptr[mid]) <= k)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void part_meta_ptr(const int32_t *__restrict__ ptr,
                                                     int32_t rows, int64_t nnz, int32_t np,
                                                     msrep_part *__restrict__ parts) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const int64_t s = (static_cast<int64_t>(i) * nnz) / np;
  const int64_t e = (static_cast<int64_t>(i + 1) * nnz) / np - 1;
  msrep_part P;
  P.start_idx = s;
  P.end_idx = e;
  if (s > e) {
    const int32_t sr = s < nnz ? row_containing(ptr, rows, s) : rows;
    P.start_row = sr;
    P.end_row = sr - 1;
    P.start_flag = 0;
    P.end_flag = 0;
    P.lptr_off = static_cast<int64_t>(sr) + 2 * static_cast<int64_t>(i);
  } else {
    const int32_t sr = row_containing(ptr, rows, s);
    const int32_t er = row_containing(ptr, rows, e);
    P.start_row = sr;
    P.end_row = er;
    P.start_flag = s > static_cast<int64_t>(ptr[sr]) ? 1 : 0;
    P.end_flag = e + 1 < static_cast<int64_t>(ptr[er + 1]) ? 1 : 0;
    P.lptr_off = static_cast<int64_t>(sr) + 2 * static_cast<int64_t>(i);
  }
  parts[i] = P;
}

// Local pointers: blocks_per_part blocks share one partition's R+1 entries.
__global__ __launch_bounds__(256) void part_lptr(const int32_t *__restrict__ ptr, int32_t np,
                                                 const msrep_part *__restrict__ parts,
                                                 int32_t *__restrict__ lptr, int64_t cap,
                                                 int32_t blocks_per_part,
                                                 int64_t *__restrict__ lptr_len) {
  const int32_t i = blockIdx.x / blocks_per_part;
  const int32_t sub = blockIdx.x % blocks_per_part;
  if (i >= np) return;
  const msrep_part P = parts[i];
  const int64_t s = P.start_idx, e = P.end_idx;
  const int64_t R = static_cast<int64_t>(P.end_row) - P.start_row + 1;  // 0 when empty
  const int64_t n_ent = R + 1;
  const int64_t per = (n_ent + blocks_per_part - 1) / blocks_per_part;
  const int64_t j_lo = sub * per;
  const int64_t j_hi = j_lo + per < n_ent ? j_lo + per : n_ent;
  for (int64_t j = j_lo + threadIdx.x; j < j_hi; j += blockDim.x) {
    const int64_t dst = P.lptr_off + j;
    if (dst < 0 || dst >= cap) continue;  // only reachable for a corrupt ptr
    int64_t v = 0;
    if (R > 0) {
      v = ptr[P.start_row + j];
      v = v < s ? s : v;
      v = v > e + 1 ? e + 1 : v;
      v -= s;
    }
    lptr[dst] = static_cast<int32_t>(v);
  }
  if (lptr_len && i == np - 1 && sub == 0 && threadIdx.x == 0) *lptr_len = P.lptr_off + n_ent;
}

// pCOO on row-sorted COO: rows come straight from row_idx.  Called with the
// column index of column-sorted COO it gives that format's records (columns
// in the row fields).
__global__ __launch_bounds__(256) void part_meta_coo(const int32_t *__restrict__ row_idx,
                                                     int32_t rows, int64_t nnz, int32_t np,
                                                     msrep_part *__restrict__ parts) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const int64_t s = (static_cast<int64_t>(i) * nnz) / np;
  const int64_t e = (static_cast<int64_t>(i + 1) * nnz) / np - 1;
  msrep_part P;
  P.start_idx = s;
  P.end_idx = e;
  P.lptr_off = 0;
  if (s > e) {
    const int32_t sr = s < nnz ? row_idx[s] : rows;
    P.start_row = sr;
    P.end_row = sr - 1;
    P.start_flag = 0;
    P.end_flag = 0;
  } else {
    P.start_row = row_idx[s];
    P.end_row = row_idx[e];
    P.start_flag = (s > 0 && row_idx[s - 1] == P.start_row) ? 1 : 0;
    P.end_flag = (e + 1 < nnz && row_idx[e + 1] == P.end_row) ? 1 : 0;
  }
  parts[i] = P;
}

// COO in any order: equal-nnz position ranges only (rows are not grouped,
// so no partition has rows of its own): start_row 0, end_row -1, flags 0.
__global__ __launch_bounds__(256) void part_meta_any(int64_t nnz, int32_t np,
                                                     msrep_part *__restrict__ parts) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  msrep_part P;
  P.start_idx = (static_cast<int64_t>(i) * nnz) / np;
  P.end_idx = (static_cast<int64_t>(i + 1) * nnz) / np - 1;
  P.start_row = 0;
  P.end_row = -1;
  P.start_flag = 0;
  P.end_flag = 0;
  P.lptr_off = 0;
  parts[i] = P;
}

// The paper's Baseline split (Sec. 5.3): partition i takes the whole rows
// (CSC: columns) floor(i*rows/np) .. floor((i+1)*rows/np) - 1, whatever
// their nonzeros; no row is split, so both flags are 0.  The record fields
// keep their equal-nnz meaning: start_row / end_row are the rows holding the
// block's first and last nonzero, and a block without nonzeros is an empty
// partition (end_idx = start_idx - 1, start_row = the row of start_idx).
__global__ __launch_bounds__(256) void part_meta_rows_ptr(const int32_t *__restrict__ ptr,
                                                          int32_t rows, int64_t nnz, int32_t np,
                                                          msrep_part *__restrict__ parts) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const int32_t r_lo = static_cast<int32_t>((static_cast<int64_t>(i) * rows) / np);
  const int32_t r_hi = static_cast<int32_t>((static_cast<int64_t>(i + 1) * rows) / np);
  const int64_t s = ptr[r_lo];
  const int64_t e = static_cast<int64_t>(ptr[r_hi]) - 1;
  msrep_part P;
  P.start_idx = s;
  P.end_idx = e;
  P.start_flag = 0;
  P.end_flag = 0;
  const int32_t sr = s < nnz ? row_containing(ptr, rows, s) : rows;
  P.start_row = sr;
  P.end_row = s > e ? sr - 1 : row_containing(ptr, rows, e);
  P.lptr_off = static_cast<int64_t>(sr) + 2 * static_cast<int64_t>(i);
  parts[i] = P;
}

// First position of a row-sorted row index array holding a row >= r (nnz
// if none).
__device__ int64_t first_row_at_least(const int32_t *__restrict__ row_idx, int64_t nnz,
                                      int32_t r) {
  int64_t lo = 0, hi = nnz;  // answer in [lo, hi]
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (row_idx[mid] < r)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void part_meta_rows_coo(const int32_t *__restrict__ row_idx,
                                                          int32_t rows, int64_t nnz, int32_t np,
                                                          msrep_part *__restrict__ parts) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const int32_t r_lo = static_cast<int32_t>((static_cast<int64_t>(i) * rows) / np);
  const int32_t r_hi = static_cast<int32_t>((static_cast<int64_t>(i + 1) * rows) / np);
  const int64_t s = first_row_at_least(row_idx, nnz, r_lo);
  const int64_t e = first_row_at_least(row_idx, nnz, r_hi) - 1;
  msrep_part P;
  P.start_idx = s;
  P.end_idx = e;
  P.start_flag = 0;
  P.end_flag = 0;
  P.lptr_off = 0;
  P.start_row = s < nnz ? row_idx[s] : rows;
  P.end_row = s > e ? P.start_row - 1 : row_idx[e];
  parts[i] = P;
}

__global__ void store_i64(int64_t *p, int64_t v) { *p = v; }

}  // namespace
}  // namespace msrep

using namespace msrep;

extern "C" int64_t msrep_lptr_bound(int32_t rows, int32_t np) {
  if (rows < 0 || np <= 0) return -1;
  return static_cast<int64_t>(rows) + 2 * static_cast<int64_t>(np);
}

namespace {

enum Split { kSplitNnz, kSplitRows };

msrep_status build_partition(const msrep_mat *A, int32_t np, msrep_part *parts_d, int32_t *lptr_d,
                             int64_t lptr_cap, int64_t *lptr_len_d, void *stream, Split split,
                             const char *who) {
  if (msrep_status st = check_mat(A, who)) return st;
  if (np <= 0) return fail(MSREP_ERR_ARG, "%s: np must be positive (got %d)", who, np);
  if (!parts_d) return fail(MSREP_ERR_ARG, "%s: parts_d is NULL", who);
  if (split == kSplitRows && A->fmt == MSREP_COO_ANY)
    return fail(MSREP_ERR_UNSUPPORTED, "%s: COO in any order has no row blocks", who);
  hipStream_t s = as_stream(stream);
  const int grid = (np + 255) / 256;
  if (A->fmt == MSREP_COO || A->fmt == MSREP_COO_ANY || A->fmt == MSREP_COO_COL) {
    // the sorted index: rows of row-sorted COO, columns of column-sorted COO
    // (Algorithm 6 applied to that index; the records then hold columns)
    const bool by_col = A->fmt == MSREP_COO_COL;
    const int32_t *key = by_col ? A->idx2 : A->idx;
    const int32_t extent = by_col ? A->n : A->m;
    if (split == kSplitRows) {
      hipLaunchKernelGGL(part_meta_rows_coo, dim3(grid), dim3(256), 0, s, key, extent, A->nnz,
                         np, parts_d);
      MSREP_LAUNCHED("part_meta_rows_coo");
    } else if (A->fmt != MSREP_COO_ANY) {
      hipLaunchKernelGGL(part_meta_coo, dim3(grid), dim3(256), 0, s, key, extent, A->nnz, np,
                         parts_d);
      MSREP_LAUNCHED("part_meta_coo");
    } else {
      hipLaunchKernelGGL(part_meta_any, dim3(grid), dim3(256), 0, s, A->nnz, np, parts_d);
      MSREP_LAUNCHED("part_meta_any");
    }
    if (lptr_len_d) {
      hipLaunchKernelGGL(store_i64, dim3(1), dim3(1), 0, s, lptr_len_d, int64_t(0));
      MSREP_LAUNCHED("store_i64");
    }
    return ok();
  }
  const int32_t rows = major_dim(A);
  const int64_t need = msrep_lptr_bound(rows, np);
  if (!lptr_d) return fail(MSREP_ERR_ARG, "%s: lptr_d is NULL", who);
  if (lptr_cap < need)
    return fail(MSREP_ERR_SIZE, "%s: lptr_cap %lld < rows + 2*np = %lld", who,
                static_cast<long long>(lptr_cap), static_cast<long long>(need));
  if (split == kSplitRows) {
    hipLaunchKernelGGL(part_meta_rows_ptr, dim3(grid), dim3(256), 0, s, A->ptr, rows, A->nnz, np,
                       parts_d);
    MSREP_LAUNCHED("part_meta_rows_ptr");
  } else {
    hipLaunchKernelGGL(part_meta_ptr, dim3(grid), dim3(256), 0, s, A->ptr, rows, A->nnz, np,
                       parts_d);
    MSREP_LAUNCHED("part_meta_ptr");
  }
  // enough blocks to cover the device even when np is small
  const int32_t bpp = np >= 2048 ? 1 : (2048 + np - 1) / np;
  hipLaunchKernelGGL(part_lptr, dim3(static_cast<unsigned>(np) * bpp), dim3(256), 0, s, A->ptr, np,
                     parts_d, lptr_d, lptr_cap, bpp, lptr_len_d);
  MSREP_LAUNCHED("part_lptr");
  return ok();
}

}  // namespace

extern "C" msrep_status msrep_build_partition(const msrep_mat *A, int32_t np, msrep_part *parts_d,
                                              int32_t *lptr_d, int64_t lptr_cap,
                                              int64_t *lptr_len_d, void *stream) {
  return build_partition(A, np, parts_d, lptr_d, lptr_cap, lptr_len_d, stream, kSplitNnz,
                         "msrep_build_partition");
}

extern "C" msrep_status msrep_build_partition_rows(const msrep_mat *A, int32_t np,
                                                   msrep_part *parts_d, int32_t *lptr_d,
                                                   int64_t lptr_cap, int64_t *lptr_len_d,
                                                   void *stream) {
  return build_partition(A, np, parts_d, lptr_d, lptr_cap, lptr_len_d, stream, kSplitRows,
                         "msrep_build_partition_rows");
}
