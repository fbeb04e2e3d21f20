// msrep_convert: CSR, CSC, row-sorted and column-sorted COO into one another
// on the GPU (msRep Sec. 2.1; CSC(A) = CSR(A^T)).  All conversions are stable and deterministic:
//   * expand:  the major index of every nonzero from a compressed pointer
//              (mark each non-empty row's first position, inclusive max-scan);
//   * compress: a pointer from sorted major indices (counting + scan);
//   * transpose: a stable LSD radix sort of (new major index, position)
//              pairs, 8-bit digits, ranks formed with wavefront ballots, so
//              entries that tie keep their storage order;
//   * gathers move indices and values (2, 4 or 8 bytes) by the permutation.
#include <algorithm>

#include "common.hpp"
#include "scan.hpp"

namespace msrep {
namespace {

using namespace scan;
constexpr int kRadix = 256;

// ------------------------------------------------------ expand/compress
template <typename T>
__global__ void fill(T *__restrict__ a, int64_t n, T v) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    a[i] = v;
}

// major index r at the first position of every non-empty major slice
__global__ void mark_starts(const int32_t *__restrict__ ptr, int32_t rows, int64_t nnz,
                            int32_t *__restrict__ out) {
  for (int64_t r = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; r < rows;
       r += int64_t(gridDim.x) * blockDim.x) {
    const int64_t a = ptr[r], b = ptr[r + 1];
    if (a < b && a >= 0 && a < nnz) out[a] = static_cast<int32_t>(r);
  }
}

// counts[i + 1] += 1 for every index i (counts has minor + 1 entries)
__global__ void histogram(const int32_t *__restrict__ idx, int64_t nnz, int32_t minor,
                          int32_t *__restrict__ counts) {
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < nnz;
       k += int64_t(gridDim.x) * blockDim.x) {
    const int32_t i = idx[k];
    if (static_cast<uint32_t>(i) < static_cast<uint32_t>(minor)) atomicAdd(counts + i + 1, 1);
  }
}

// ptr of a row-sorted COO: ptr[r] = first position whose row is >= r
__global__ void rows_to_ptr(const int32_t *__restrict__ row, int64_t nnz, int32_t m,
                            int32_t *__restrict__ ptr) {
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k <= nnz;
       k += int64_t(gridDim.x) * blockDim.x) {
    int64_t lo = k == 0 ? 0 : static_cast<int64_t>(row[k - 1]) + 1;
    int64_t hi = k == nnz ? m : static_cast<int64_t>(row[k]);
    lo = lo < 0 ? 0 : lo;
    hi = hi > m ? m : hi;
    for (int64_t r = lo; r <= hi; ++r) ptr[r] = static_cast<int32_t>(k);
  }
}

// --------------------------------------------------- LSD radix sort
__global__ void iota(int32_t *__restrict__ a, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    a[i] = static_cast<int32_t>(i);
}

// hist[d * nb + b] = number of keys of tile b whose digit is d
__global__ __launch_bounds__(kBlock) void radix_hist(const uint32_t *__restrict__ keys, int64_t n,
                                                     int shift, int64_t nb,
                                                     int32_t *__restrict__ hist) {
  __shared__ int32_t cnt[kRadix];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = blockIdx.x * int64_t(kTile);
  for (int i = 0; i < kItems; ++i) {
    const int64_t k = base + i * kBlock + threadIdx.x;
    if (k < n) atomicAdd(&cnt[(keys[k] >> shift) & (kRadix - 1)], 1);
  }
  __syncthreads();
  hist[threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter: tile items are taken in storage order (round i holds items
// i*256 + tid); an item's rank is the number of earlier tile items with its
// digit, found with ballots inside a wavefront and LDS counts across them.
__global__ __launch_bounds__(kBlock) void radix_scatter(
    const uint32_t *__restrict__ kin, const int32_t *__restrict__ vin, int64_t n, int shift,
    int64_t nb, const int32_t *__restrict__ off, uint32_t *__restrict__ kout,
    int32_t *__restrict__ vout) {
  __shared__ int32_t run[kRadix];
  __shared__ int32_t wcnt[kBlock / 64][kRadix];
  __shared__ int32_t base_off[kRadix];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  run[tid] = 0;
  base_off[tid] = off[tid * nb + blockIdx.x];
  for (int i = 0; i < kBlock / 64; ++i) wcnt[i][tid] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = blockIdx.x * int64_t(kTile);
  for (int i = 0; i < kItems; ++i) {
    const int64_t k = base + i * kBlock + tid;
    const bool valid = k < n;
    const uint32_t key = valid ? kin[k] : 0u;
    const int32_t val = valid ? vin[k] : 0;
    const int d = static_cast<int>((key >> shift) & (kRadix - 1));
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bal = __ballot((d >> b) & 1);
      peers &= ((d >> b) & 1) ? bal : ~bal;
    }
    const int wrank = __popcll(peers & lt);
    if (valid && wrank == 0) wcnt[w][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int32_t r = run[d] + wrank;
      for (int v = 0; v < w; ++v) r += wcnt[v][d];
      const int64_t dst = static_cast<int64_t>(base_off[d]) + r;
      kout[dst] = key;
      vout[dst] = val;
    }
    __syncthreads();
    int32_t add = 0;
    for (int v = 0; v < kBlock / 64; ++v) {
      add += wcnt[v][tid];
      wcnt[v][tid] = 0;
    }
    run[tid] += add;
    __syncthreads();
  }
}

// ---------------------------------------------------------- gathers
template <typename E>
__global__ void gather(const E *__restrict__ src, const int32_t *__restrict__ perm, int64_t n,
                       E *__restrict__ dst) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    dst[i] = src[perm[i]];
}

int grid_for(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return static_cast<int>(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

// ----------------------------------------------------- workspace plan
struct Ws {
  int32_t *major;          // nnz: major index of every source entry
  uint32_t *ka, *kb;       // nnz: radix keys
  int32_t *va, *vb;        // nnz: radix values (positions)
  int32_t *hist;           // 256 * tiles(nnz)
  int32_t *agg;            // tiles(max(nnz, 256*tiles, minor+1)) scan aggregates
  int64_t *agg64;
  size_t bytes;
};

Ws plan_ws(void *base, int64_t nnz, int64_t minor) {
  Ws w{};
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o += align_up(b, 256);
    return base ? static_cast<char *>(base) + at : nullptr;
  };
  const int64_t nt = tiles(nnz);
  const int64_t hist_n = kRadix * nt;
  const int64_t scan_n = std::max<int64_t>({nnz, hist_n, minor + 1, 1});
  w.major = reinterpret_cast<int32_t *>(take(4 * static_cast<size_t>(nnz)));
  w.ka = reinterpret_cast<uint32_t *>(take(4 * static_cast<size_t>(nnz)));
  w.kb = reinterpret_cast<uint32_t *>(take(4 * static_cast<size_t>(nnz)));
  w.va = reinterpret_cast<int32_t *>(take(4 * static_cast<size_t>(nnz)));
  w.vb = reinterpret_cast<int32_t *>(take(4 * static_cast<size_t>(nnz)));
  w.hist = reinterpret_cast<int32_t *>(take(4 * static_cast<size_t>(hist_n)));
  w.agg = reinterpret_cast<int32_t *>(take(4 * static_cast<size_t>(tiles(scan_n) + 1)));
  w.agg64 = nullptr;
  w.bytes = o;
  return w;
}

// Major index (row of CSR, column of CSC) of every entry.
msrep_status expand(const int32_t *ptr, int32_t rows, int64_t nnz, int32_t *out, int32_t *agg,
                    hipStream_t s) {
  if (nnz == 0) return MSREP_OK;
  hipLaunchKernelGGL(fill<int32_t>, dim3(grid_for(nnz)), dim3(256), 0, s, out, nnz, int32_t(-1));
  MSREP_LAUNCHED("fill");
  hipLaunchKernelGGL(mark_starts, dim3(grid_for(rows)), dim3(256), 0, s, ptr, rows, nnz, out);
  MSREP_LAUNCHED("mark_starts");
  return device_scan<int32_t, MaxOp>(out, out, nnz, agg, true, s);
}

// Pointer of minor+1 entries from unsorted indices: counts, then a scan.
msrep_status compress_counts(const int32_t *idx, int64_t nnz, int32_t minor, int32_t *ptr,
                             int32_t *agg, hipStream_t s) {
  hipLaunchKernelGGL(fill<int32_t>, dim3(grid_for(minor + 1)), dim3(256), 0, s, ptr,
                     int64_t(minor) + 1, int32_t(0));
  MSREP_LAUNCHED("fill");
  if (nnz > 0) {
    hipLaunchKernelGGL(histogram, dim3(grid_for(nnz)), dim3(256), 0, s, idx, nnz, minor, ptr);
    MSREP_LAUNCHED("histogram");
  }
  return device_scan<int32_t, SumOp>(ptr, ptr, int64_t(minor) + 1, agg, true, s);
}

// Stable sort of positions 0..nnz-1 by key (keys < 2^bits); returns the
// buffer holding the permutation and the sorted keys.
msrep_status stable_sort(const int32_t *keys, int64_t nnz, int bits, Ws &w, hipStream_t s,
                         int32_t **perm, uint32_t **sorted) {
  uint32_t *kin = w.ka, *kout = w.kb;
  int32_t *vin = w.va, *vout = w.vb;
  MSREP_HIP(hipMemcpyAsync(kin, keys, 4 * static_cast<size_t>(nnz), hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(iota, dim3(grid_for(nnz)), dim3(256), 0, s, vin, nnz);
  MSREP_LAUNCHED("iota");
  const int64_t nt = tiles(nnz);
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(radix_hist, dim3(nt), dim3(kBlock), 0, s, kin, nnz, shift, nt, w.hist);
    MSREP_LAUNCHED("radix_hist");
    if (msrep_status st = device_scan<int32_t, SumOp>(w.hist, w.hist, kRadix * nt, w.agg, false, s))
      return st;
    hipLaunchKernelGGL(radix_scatter, dim3(nt), dim3(kBlock), 0, s, kin, vin, nnz, shift, nt,
                       w.hist, kout, vout);
    MSREP_LAUNCHED("radix_scatter");
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
  *perm = vin;
  *sorted = kin;
  return MSREP_OK;
}

int key_bits(int64_t range) {
  int b = 1;
  while (b < 32 && (int64_t(1) << b) < range) ++b;
  return b;
}

msrep_status gather_values(const void *src, const int32_t *perm, int64_t nnz, int32_t vtype,
                           void *dst, hipStream_t s) {
  const int g = grid_for(nnz);
  switch (value_bytes(vtype)) {
    case 8:
      hipLaunchKernelGGL(gather<uint64_t>, dim3(g), dim3(256), 0, s,
                         static_cast<const uint64_t *>(src), perm, nnz, static_cast<uint64_t *>(dst));
      break;
    case 4:
      hipLaunchKernelGGL(gather<uint32_t>, dim3(g), dim3(256), 0, s,
                         static_cast<const uint32_t *>(src), perm, nnz, static_cast<uint32_t *>(dst));
      break;
    default:
      hipLaunchKernelGGL(gather<uint16_t>, dim3(g), dim3(256), 0, s,
                         static_cast<const uint16_t *>(src), perm, nnz, static_cast<uint16_t *>(dst));
  }
  MSREP_LAUNCHED("gather");
  return MSREP_OK;
}

}  // namespace
}  // namespace msrep

using namespace msrep;

extern "C" size_t msrep_convert_ws_bytes(const msrep_mat *src, int32_t dst_fmt) {
  if (!src || src->nnz < 0 || src->m < 0 || src->n < 0) return 0;
  (void)dst_fmt;
  const int64_t minor = std::max(src->m, src->n);
  return plan_ws(nullptr, src->nnz, minor).bytes;
}

namespace {

// Row-major formats (CSR, row-sorted COO) keep their nonzeros grouped by
// row, column-major ones (CSC, column-sorted COO) by column.
bool row_major(int32_t fmt) { return fmt == MSREP_CSR || fmt == MSREP_COO; }
bool compressed(int32_t fmt) { return fmt == MSREP_CSR || fmt == MSREP_CSC; }

// A format's index arrays in terms of its own order: the major index (the
// one it is grouped by: row for CSR / COO, column for CSC / COO_COL), either
// compressed (ptr) or one per nonzero (exp), and the minor index.
struct Sides {
  const int32_t *ptr, *exp, *minor;
  int32_t major_extent, minor_extent;
};

Sides sides_of(const msrep_mat *A) {
  const bool rm = row_major(A->fmt);
  Sides d{};
  d.major_extent = rm ? A->m : A->n;
  d.minor_extent = rm ? A->n : A->m;
  switch (A->fmt) {
    case MSREP_CSR:
    case MSREP_CSC: d.ptr = A->ptr; d.minor = A->idx; break;
    case MSREP_COO: d.exp = A->idx; d.minor = A->idx2; break;
    default: d.exp = A->idx2; d.minor = A->idx; break;  // MSREP_COO_COL
  }
  return d;
}

// Where the destination's major (expanded) and minor indices go.
int32_t *dst_exp(msrep_mat *D) {
  return const_cast<int32_t *>(D->fmt == MSREP_COO ? D->idx : D->idx2);
}
int32_t *dst_minor(msrep_mat *D) {
  return const_cast<int32_t *>(D->fmt == MSREP_COO ? D->idx2 : D->idx);
}

}  // namespace

extern "C" msrep_status msrep_convert(const msrep_mat *src, msrep_mat *dst, void *ws_d,
                                      size_t ws_bytes, void *stream) {
  if (msrep_status st = check_mat(src, "msrep_convert")) return st;
  if (!dst) return fail(MSREP_ERR_ARG, "msrep_convert: dst is NULL");
  if (dst->fmt < MSREP_CSR || dst->fmt > MSREP_COO_COL)
    return fail(MSREP_ERR_ARG, "msrep_convert: unknown target format %d", dst->fmt);
  if (src->fmt == MSREP_COO_ANY || dst->fmt == MSREP_COO_ANY)
    return fail(MSREP_ERR_UNSUPPORTED,
                "msrep_convert: COO in any order is taken by msrep_spmv as it is, not converted");
  if (dst->m != src->m || dst->n != src->n || dst->nnz != src->nnz || dst->vtype != src->vtype)
    return fail(MSREP_ERR_ARG, "msrep_convert: dst shape/nnz/vtype differ from src");
  const int64_t nnz = src->nnz;
  const bool dcomp = compressed(dst->fmt);
  int32_t *dptr = const_cast<int32_t *>(dst->ptr);
  void *dval = const_cast<void *>(dst->val);
  if (dcomp && !dptr) return fail(MSREP_ERR_ARG, "msrep_convert: dst ptr is NULL");
  if (nnz > 0 && (!dst->idx || !dval || (!dcomp && !dst->idx2)))
    return fail(MSREP_ERR_ARG, "msrep_convert: dst arrays are NULL");
  const size_t need = msrep_convert_ws_bytes(src, dst->fmt);
  if (!ws_d || ws_bytes < need)
    return fail(MSREP_ERR_SIZE, "msrep_convert: workspace of %zu bytes needed (got %zu)", need,
                ws_d ? ws_bytes : size_t(0));
  hipStream_t s = as_stream(stream);
  Ws w = plan_ws(ws_d, nnz, std::max(src->m, src->n));
  const size_t vb = static_cast<size_t>(value_bytes(src->vtype)) * nnz;
  const Sides S = sides_of(src);
  int32_t *dminor = dst_minor(dst);

  if (row_major(src->fmt) == row_major(dst->fmt)) {
    // same grouping: the major index is compressed or expanded, the minor
    // index and the values are copied
    if (dcomp) {
      if (S.ptr)
        MSREP_HIP(hipMemcpyAsync(dptr, S.ptr, 4 * (static_cast<size_t>(S.major_extent) + 1),
                                 hipMemcpyDeviceToDevice, s));
      else {
        hipLaunchKernelGGL(rows_to_ptr, dim3(grid_for(nnz + 1)), dim3(256), 0, s, S.exp, nnz,
                           S.major_extent, dptr);
        MSREP_LAUNCHED("rows_to_ptr");
      }
    } else if (nnz > 0) {
      if (S.ptr) {
        if (msrep_status st = expand(S.ptr, S.major_extent, nnz, dst_exp(dst), w.agg, s))
          return st;
      } else {
        MSREP_HIP(hipMemcpyAsync(dst_exp(dst), S.exp, 4 * nnz, hipMemcpyDeviceToDevice, s));
      }
    }
    if (nnz > 0) {
      MSREP_HIP(hipMemcpyAsync(dminor, S.minor, 4 * nnz, hipMemcpyDeviceToDevice, s));
      MSREP_HIP(hipMemcpyAsync(dval, src->val, vb, hipMemcpyDeviceToDevice, s));
    }
    return ok();
  }
  // the transposing conversions: a stable sort of the positions by the
  // source's minor index (the destination's major one); the source's major
  // index becomes the destination's minor one
  const int32_t *key = S.minor;
  const int32_t key_range = S.minor_extent;
  const int32_t *other = S.exp;
  if (S.ptr) {
    if (msrep_status st = expand(S.ptr, S.major_extent, nnz, w.major, w.agg, s)) return st;
    other = w.major;
  }
  if (dcomp) {
    if (msrep_status st = compress_counts(key, nnz, key_range, dptr, w.agg, s)) return st;
  }
  if (nnz == 0) return ok();
  int32_t *perm = nullptr;
  uint32_t *sorted = nullptr;
  if (msrep_status st = stable_sort(key, nnz, key_bits(key_range), w, s, &perm, &sorted)) return st;
  if (!dcomp)
    MSREP_HIP(hipMemcpyAsync(dst_exp(dst), sorted, 4 * nnz, hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(gather<int32_t>, dim3(grid_for(nnz)), dim3(256), 0, s, other, perm, nnz,
                     dminor);
  MSREP_LAUNCHED("gather");
  if (msrep_status st = gather_values(src->val, perm, nnz, src->vtype, dval, s)) return st;
  return ok();
}
