// msrep_convert: CSR, CSC, row-sorted and column-sorted COO into one another
// on the GPU (msRep Sec. 2.1; CSC(A) = CSR(A^T)).  All conversions are stable and deterministic:
//   * expand:  the major index of every nonzero from a compressed pointer
//              (per tile of positions: the row holding its first position by
//              binary search, the rows starting inside it marked in LDS, a
//              block max-scan carrying each mark forward);
//   * compress: a pointer from sorted major indices (each position writes the
//              pointers of the indices it starts);
//   * transpose: a stable LSD radix sort of the entries by their new major
//              index, 8-bit digits, ranks formed with wavefront ballots, so
//              entries that tie keep their storage order; each entry's new
//              minor index and value (2, 4 or 8 bytes) travel with its key,
//              the first pass reading the source's arrays and the last one
//              writing the destination's, and each XCD sorts a contiguous
//              run of tiles, so the short per-digit runs of neighbouring
//              tiles meet in one L2;
//   * COO in any order: two stable sorts of (key, position) pairs, then
//              gathers that move the minor indices and the values by the
//              permutation.
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

// The last row r in [0, rows) with ptr[r] <= key, found by one wavefront:
// each step probes 64 evenly spaced rows of the interval left.
__device__ int32_t wave_row_of(const int32_t *__restrict__ ptr, int32_t rows, int64_t key) {
  const int lane = threadIdx.x & 63;
  int64_t lo = 0, hi = rows;
  while (hi - lo > 1) {
    const int64_t step = (hi - lo + 63) / 64;
    const int64_t r = lo + lane * step;
    const uint64_t le = __ballot(r < hi && ptr[r] <= key);
    const int j = le ? 63 - __clzll(static_cast<long long>(le)) : 0;
    lo += j * step;
    hi = lo + step < hi ? lo + step : hi;
  }
  return static_cast<int32_t>(lo);
}

// Expanded major indices of one tile of kTile positions.  ptr must be
// non-decreasing from ptr[0] = 0 to ptr[rows] = nnz (a malformed pointer gives
// wrong indices but no access outside ptr, out or LDS).
__global__ __launch_bounds__(kBlock) void expand_tile(const int32_t *__restrict__ ptr,
                                                      int32_t rows, int64_t nnz,
                                                      int32_t *__restrict__ out) {
  constexpr int kPad = kTile + kTile / 32;  // one pad word per 32: conflict-free strided reads
  __shared__ int32_t mark[kPad];
  __shared__ int32_t ends[2];
  __shared__ int32_t sh[kBlock / 64];
  const int tid = threadIdx.x;
  const int64_t base = blockIdx.x * int64_t(kTile);
  const int64_t last = (base + kTile < nnz ? base + kTile : nnz) - 1;
  if (tid < 128) {  // wavefronts 0 and 1: the rows of the first and last positions
    const int32_t r = wave_row_of(ptr, rows, tid < 64 ? base : last);
    if ((tid & 63) == 0) ends[tid >> 6] = r;
  }
  for (int i = tid; i < kPad; i += kBlock) mark[i] = -1;
  __syncthreads();
  const int32_t r0 = ends[0], r1 = ends[1];
  if (tid == 0) mark[0] = r0;
  // rows starting inside the tile; of several rows starting at one position
  // (empty rows before it) the last one marks it
  for (int32_t r = r0 + 1 + tid; r <= r1; r += kBlock) {
    const int64_t a = ptr[r];
    if (a > base && a <= last && ptr[r + 1] != a) {
      const int i = static_cast<int>(a - base);
      mark[i + i / 32] = r;
    }
  }
  __syncthreads();
  int32_t run = -1;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int i = tid * kItems + j;
    run = max(run, mark[i + i / 32]);
  }
  int32_t before;
  block_exscan<int32_t, MaxOp>(run, before, sh);
  run = before;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int i = tid * kItems + j;
    run = max(run, mark[i + i / 32]);
    mark[i + i / 32] = run;
  }
  __syncthreads();
  for (int i = tid; i < kTile; i += kBlock)
    if (base + i <= last) out[base + i] = mark[i + i / 32];
}

// ptr of a row-sorted COO: ptr[r] = first position whose row is >= r.
// Thread t takes positions 4t .. 4t+3 (and nnz itself, for the rows after
// the last entry): position k writes the pointers of the rows from the one
// after row[k-1] up to row[k].
__global__ void rows_to_ptr(const int32_t *__restrict__ row, int64_t nnz, int32_t m,
                            int32_t *__restrict__ ptr) {
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; 4 * t <= nnz;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t k0 = 4 * t;
    int64_t prev = k0 == 0 ? -1 : static_cast<int64_t>(row[k0 - 1]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t k = k0 + i;
      if (k > nnz) break;
      const int64_t cur = k == nnz ? m : static_cast<int64_t>(row[k]);
      const int64_t lo = prev + 1 < 0 ? 0 : prev + 1;
      const int64_t hi = cur > m ? m : cur;
      for (int64_t r = lo; r <= hi; ++r) ptr[r] = static_cast<int32_t>(k);
      prev = cur;
    }
  }
}

// Threads of rows_to_ptr for nnz positions.
int grid_for_ptr(int64_t nnz) {
  const int64_t g = (nnz / 4 + 1 + 255) / 256;
  return static_cast<int>(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

// --------------------------------------------------- LSD radix sort
// hist[d * nb + b] = number of keys of tile b whose digit is d
__global__ __launch_bounds__(kBlock) void radix_hist(const uint32_t *__restrict__ keys, int64_t n,
                                                     int shift, int64_t nb,
                                                     int32_t *__restrict__ hist) {
  __shared__ int32_t cnt[kRadix];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  const int64_t base = tile * int64_t(kTile);
  for (int i = 0; i < kItems; ++i) {
    const int64_t k = base + i * kBlock + threadIdx.x;
    if (k < n) atomicAdd(&cnt[(keys[k] >> shift) & (kRadix - 1)], 1);
  }
  __syncthreads();
  hist[threadIdx.x * nb + tile] = cnt[threadIdx.x];
}

// Destinations of the items of one tile for the digit at `shift` (a stable
// scatter).  Wavefront w takes the w-th quarter of the tile, in rounds of 64
// items in storage order.  Every item is ranked among the earlier items of
// its quarter with the same digit (ballots within a round, per-wavefront LDS
// counts across rounds); the quarters' counts are then combined per digit,
// and each item goes to the tile's offset for its digit + the earlier
// quarters' counts + its rank.  dst[i] is defined for the items below n.
constexpr int kSortWaves = kBlock / 64, kQuarter = kTile / kSortWaves, kRounds = kQuarter / 64;

__device__ __forceinline__ void tile_destinations(const uint32_t (&key)[kRounds], int64_t base,
                                                  int64_t n, int shift, int64_t nb, int tile,
                                                  const int32_t *__restrict__ off,
                                                  int32_t (*wcnt)[kRadix],
                                                  int32_t (&dst)[kRounds]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int v = 0; v < kSortWaves; ++v) wcnt[v][tid] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int i = 0; i < kRounds; ++i) {
    const bool valid = base + i * 64 < n;
    const int d = static_cast<int>((key[i] >> shift) & (kRadix - 1));
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bal = __ballot((d >> b) & 1);
      peers &= ((d >> b) & 1) ? bal : ~bal;
    }
    const int wrank = __popcll(peers & lt);
    const int32_t c = wcnt[w][d];
    dst[i] = c + wrank;
    wave_lds_sync();
    if (valid && wrank == 0) wcnt[w][d] = c + __popcll(peers);
    wave_lds_sync();
  }
  __syncthreads();
  {  // digit tid: where each quarter's items of this digit start
    int32_t o = off[tid * nb + tile];
    for (int v = 0; v < kSortWaves; ++v) {
      const int32_t c = wcnt[v][tid];
      wcnt[v][tid] = o;
      o += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kRounds; ++i)
    dst[i] += wcnt[w][static_cast<int>((key[i] >> shift) & (kRadix - 1))];
}

// Stable scatter of one tile of (key, position) pairs.
// kIota: the values are the positions themselves (vin is not read).
template <bool kIota>
__global__ __launch_bounds__(kBlock) void radix_scatter(
    const uint32_t *__restrict__ kin, const int32_t *__restrict__ vin, int64_t n, int shift,
    int64_t nb, const int32_t *__restrict__ off, uint32_t *__restrict__ kout,
    int32_t *__restrict__ vout, const int32_t *__restrict__ mode, int32_t want) {
  if (mode && *mode != want) return;
  __shared__ int32_t wcnt[kSortWaves][kRadix];
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  const int64_t base = tile * int64_t(kTile) + (threadIdx.x >> 6) * int64_t(kQuarter) +
                       (threadIdx.x & 63);
  uint32_t key[kRounds];
  int32_t val[kRounds], dst[kRounds];
#pragma unroll
  for (int i = 0; i < kRounds; ++i) {
    const int64_t k = base + i * 64;
    const bool valid = k < n;
    key[i] = valid ? kin[k] : 0u;
    val[i] = kIota ? static_cast<int32_t>(k) : (valid ? vin[k] : 0);
  }
  tile_destinations(key, base, n, shift, nb, tile, off, wcnt, dst);
#pragma unroll
  for (int i = 0; i < kRounds; ++i) {
    if (base + i * 64 < n) {
      kout[dst[i]] = key[i];
      vout[dst[i]] = val[i];
    }
  }
}

// Stable scatter of one tile of whole entries: the key (the destination's
// major index) with the destination's minor index and the value, so that
// the last pass of a transposing conversion writes the destination's arrays
// directly, with no gather by a permutation after the sort.
template <typename E>
__global__ __launch_bounds__(kBlock) void radix_scatter_entries(
    const uint32_t *__restrict__ kin, const int32_t *__restrict__ min_in,
    const E *__restrict__ vin, int64_t n, int shift, int64_t nb, const int32_t *__restrict__ off,
    uint32_t *__restrict__ kout, int32_t *__restrict__ min_out, E *__restrict__ vout,
    const int32_t *__restrict__ mode, int32_t want) {
  if (mode && *mode != want) return;
  __shared__ int32_t wcnt[kSortWaves][kRadix];
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  const int64_t base = tile * int64_t(kTile) + (threadIdx.x >> 6) * int64_t(kQuarter) +
                       (threadIdx.x & 63);
  uint32_t key[kRounds];
  int32_t mi[kRounds], dst[kRounds];
  E v[kRounds];
#pragma unroll
  for (int i = 0; i < kRounds; ++i) {
    const int64_t k = base + i * 64;
    const bool valid = k < n;
    key[i] = valid ? kin[k] : 0u;
    mi[i] = valid ? min_in[k] : 0;
    v[i] = valid ? vin[k] : E(0);
  }
  tile_destinations(key, base, n, shift, nb, tile, off, wcnt, dst);
#pragma unroll
  for (int i = 0; i < kRounds; ++i) {
    if (base + i * 64 < n) {
      kout[dst[i]] = key[i];
      min_out[dst[i]] = mi[i];
      vout[dst[i]] = v[i];
    }
  }
}

// ------------------------------------------------- transposing strategy
// A transposing conversion either sorts (key, position) pairs and then
// gathers the minor indices and values by the permutation, or moves whole
// entries through every pass of the sort.  The gathers read the source in
// destination order: a few sequential streams when the matrix is banded (a
// column's rows are near each other and near the next column's), random
// reads otherwise, where moving the entries costs less.  band_count counts,
// over every stride-th entry, those whose row and column differ by at most
// `band`; set_mode picks the pairs (0) when at least 9 in 10 do, else the
// entries (1).  Both run on the device, so the conversion stays
// asynchronous: every kernel of the unused strategy returns at once.
__global__ void band_count(const int32_t *__restrict__ a, const int32_t *__restrict__ b, int64_t n,
                           int64_t stride, int32_t band, int32_t *__restrict__ cnt) {
  int32_t c = 0;
  const int64_t step = int64_t(gridDim.x) * blockDim.x * stride;
  for (int64_t i = (blockIdx.x * int64_t(blockDim.x) + threadIdx.x) * stride; i < n; i += step) {
    const int64_t d = static_cast<int64_t>(a[i]) - b[i];
    c += (d <= band && d >= -band) ? 1 : 0;
  }
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(cnt, c);
}

// cnt_mode[0]: the count; cnt_mode[1]: the strategy
__global__ void set_mode(int32_t *__restrict__ cnt_mode, int64_t samples) {
  if (threadIdx.x == 0 && blockIdx.x == 0)
    cnt_mode[1] = static_cast<int64_t>(cnt_mode[0]) * 10 >= samples * 9 ? 0 : 1;
}

// ---------------------------------------------------------- gathers
// dst[i] = src[perm[i]].  The minor indices and the values are gathered by
// two launches: one pass over two arrays of random reads was slower.
template <typename E>
__global__ void gather(const E *__restrict__ src, const int32_t *__restrict__ perm, int64_t n,
                       E *__restrict__ dst, const int32_t *__restrict__ mode, int32_t want) {
  if (mode && *mode != want) return;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    dst[i] = src[perm[i]];
}

int grid_for(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return static_cast<int>(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

// Row-major formats (CSR, row-sorted COO) keep their nonzeros grouped by
// row, column-major ones (CSC, column-sorted COO) by column.
bool row_major(int32_t fmt) { return fmt == MSREP_CSR || fmt == MSREP_COO; }
bool compressed(int32_t fmt) { return fmt == MSREP_CSR || fmt == MSREP_CSC; }

// A conversion between a sorted format and one grouped the other way.
bool transposing(int32_t src_fmt, int32_t dst_fmt) {
  return src_fmt != MSREP_COO_ANY && row_major(src_fmt) != row_major(dst_fmt);
}

// ----------------------------------------------------- workspace plan
struct Ws {
  int32_t *major;          // nnz: major index of every source entry
  uint32_t *ka, *kb;       // nnz: radix keys
  int32_t *va, *vb;        // nnz: radix values (positions)
  int32_t *p1;             // nnz (COO in any order): positions sorted by the minor index
  void *vv;                // nnz values (transposing conversions): the sort's values between passes
  int32_t *cnt_mode;       // 2 (transposing conversions): band count and strategy
  int32_t *hist;           // 256 * tiles(nnz)
  int32_t *agg;            // tiles(256 * tiles(nnz)) scan aggregates of the histograms
  int64_t *agg64;
  size_t bytes;
};

Ws plan_ws(void *base, int64_t nnz, int64_t minor, bool any_order, size_t entry_vbytes) {
  Ws w{};
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o += align_up(b, 256);
    return base ? static_cast<char *>(base) + at : nullptr;
  };
  const int64_t nt = tiles(nnz);
  const int64_t hist_n = kRadix * nt;
  const int64_t scan_n = std::max<int64_t>(hist_n, 1);
  w.major = reinterpret_cast<int32_t *>(take(4 * static_cast<size_t>(nnz)));
  w.ka = reinterpret_cast<uint32_t *>(take(4 * static_cast<size_t>(nnz)));
  w.kb = reinterpret_cast<uint32_t *>(take(4 * static_cast<size_t>(nnz)));
  w.va = reinterpret_cast<int32_t *>(take(4 * static_cast<size_t>(nnz)));
  w.vb = reinterpret_cast<int32_t *>(take(4 * static_cast<size_t>(nnz)));
  w.p1 = any_order ? reinterpret_cast<int32_t *>(take(4 * static_cast<size_t>(nnz))) : nullptr;
  w.vv = entry_vbytes ? take(entry_vbytes * static_cast<size_t>(nnz)) : nullptr;
  w.cnt_mode = entry_vbytes ? reinterpret_cast<int32_t *>(take(8)) : nullptr;
  w.hist = reinterpret_cast<int32_t *>(take(4 * static_cast<size_t>(hist_n)));
  w.agg = reinterpret_cast<int32_t *>(take(4 * static_cast<size_t>(tiles(scan_n) + 1)));
  w.agg64 = nullptr;
  w.bytes = o;
  return w;
}

// Major index (row of CSR, column of CSC) of every entry.
msrep_status expand(const int32_t *ptr, int32_t rows, int64_t nnz, int32_t *out, hipStream_t s) {
  if (nnz == 0) return MSREP_OK;
  hipLaunchKernelGGL(expand_tile, dim3(tiles(nnz)), dim3(kBlock), 0, s, ptr, rows, nnz, out);
  MSREP_LAUNCHED("expand_tile");
  return MSREP_OK;
}

// Stable sort of positions 0..nnz-1 by key (keys < 2^bits); returns the
// buffer holding the permutation and the sorted keys.
msrep_status stable_sort(const int32_t *keys, int64_t nnz, int bits, Ws &w, hipStream_t s,
                         int32_t **perm, uint32_t **sorted) {
  // the first pass reads the source keys and positions 0..nnz-1 implicitly
  const uint32_t *kin = reinterpret_cast<const uint32_t *>(keys);
  const int32_t *vin = nullptr;
  uint32_t *kout = w.ka, *kspare = w.kb;
  int32_t *vout = w.va, *vspare = w.vb;
  const int64_t nt = tiles(nnz);
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(radix_hist, dim3(nt), dim3(kBlock), 0, s, kin, nnz, shift, nt, w.hist);
    MSREP_LAUNCHED("radix_hist");
    if (msrep_status st = device_scan<int32_t, SumOp>(w.hist, w.hist, kRadix * nt, w.agg, false, s))
      return st;
    if (vin)
      hipLaunchKernelGGL(radix_scatter<false>, dim3(nt), dim3(kBlock), 0, s, kin, vin, nnz, shift,
                         nt, w.hist, kout, vout, nullptr, 0);
    else
      hipLaunchKernelGGL(radix_scatter<true>, dim3(nt), dim3(kBlock), 0, s, kin, vin, nnz, shift,
                         nt, w.hist, kout, vout, nullptr, 0);
    MSREP_LAUNCHED("radix_scatter");
    kin = kout;
    vin = vout;
    std::swap(kout, kspare);
    std::swap(vout, vspare);
  }
  *perm = const_cast<int32_t *>(vin);
  *sorted = const_cast<uint32_t *>(kin);
  return MSREP_OK;
}

// The transposing conversions' stable sort by key (keys < 2^bits), in the
// strategy *mode picks (see band_count): either whole entries (the key, the
// minor index from min_src and the value) move through every pass, the last
// writing the minor indices into dminor and the values into dval (a pass's
// output goes to the destination arrays or to the workspace, alternately,
// so that the last one lands in the destination); or (key, position) pairs
// are sorted and the minor indices and values gathered by the permutation.
// Both sorts order the keys alike, so the histograms and the key buffers are
// shared.  Returns the buffer holding the sorted keys.
template <typename E>
msrep_status transpose_sort_t(const int32_t *keys, const int32_t *min_src, const E *val_src,
                              int64_t nnz, int bits, Ws &w, int32_t *dminor, E *dval,
                              hipStream_t s, uint32_t **sorted) {
  const int passes = (bits + 7) / 8;
  const uint32_t *kin = reinterpret_cast<const uint32_t *>(keys);
  const int32_t *min_in = min_src;
  const E *vin = val_src;
  const int32_t *pin = nullptr;  // the pairs' positions (none before the first pass)
  uint32_t *kout = w.ka, *kspare = w.kb;
  int32_t *pout = w.va, *pspare = w.vb;
  const int64_t nt = tiles(nnz);
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    const bool to_dst = (passes - 1 - p) % 2 == 0;
    int32_t *min_out = to_dst ? dminor : w.va;
    E *vout = to_dst ? dval : static_cast<E *>(w.vv);
    hipLaunchKernelGGL(radix_hist, dim3(nt), dim3(kBlock), 0, s, kin, nnz, shift, nt, w.hist);
    MSREP_LAUNCHED("radix_hist");
    if (msrep_status st = device_scan<int32_t, SumOp>(w.hist, w.hist, kRadix * nt, w.agg, false, s))
      return st;
    hipLaunchKernelGGL(radix_scatter_entries<E>, dim3(nt), dim3(kBlock), 0, s, kin, min_in, vin,
                       nnz, shift, nt, w.hist, kout, min_out, vout, w.cnt_mode + 1, 1);
    MSREP_LAUNCHED("radix_scatter_entries");
    if (pin)
      hipLaunchKernelGGL(radix_scatter<false>, dim3(nt), dim3(kBlock), 0, s, kin, pin, nnz, shift,
                         nt, w.hist, kout, pout, w.cnt_mode + 1, 0);
    else
      hipLaunchKernelGGL(radix_scatter<true>, dim3(nt), dim3(kBlock), 0, s, kin, pin, nnz, shift,
                         nt, w.hist, kout, pout, w.cnt_mode + 1, 0);
    MSREP_LAUNCHED("radix_scatter");
    kin = kout;
    min_in = min_out;
    vin = vout;
    pin = pout;
    std::swap(kout, kspare);
    std::swap(pout, pspare);
  }
  // the pairs' strategy: the entries by the permutation
  const int g = grid_for(nnz);
  hipLaunchKernelGGL(gather<int32_t>, dim3(g), dim3(256), 0, s, min_src, pin, nnz, dminor,
                     w.cnt_mode + 1, 0);
  hipLaunchKernelGGL(gather<E>, dim3(g), dim3(256), 0, s, val_src, pin, nnz, dval, w.cnt_mode + 1,
                     0);
  MSREP_LAUNCHED("gather");
  *sorted = const_cast<uint32_t *>(kin);
  return MSREP_OK;
}

// The strategy, then the sort.  keys: the source's minor index (the
// destination's major one); min_src: the source's major index (the
// destination's minor one); band: the row-column distance that counts as
// banded.
msrep_status transpose_sort(const int32_t *keys, const int32_t *min_src, const void *val_src,
                            int32_t vtype, int64_t nnz, int bits, int32_t band, Ws &w,
                            int32_t *dminor, void *dval, hipStream_t s, uint32_t **sorted) {
  const int64_t stride = std::max<int64_t>(1, nnz / 65536);
  const int64_t samples = (nnz + stride - 1) / stride;
  hipLaunchKernelGGL(fill<int32_t>, dim3(1), dim3(64), 0, s, w.cnt_mode, int64_t(2), int32_t(0));
  hipLaunchKernelGGL(band_count, dim3(static_cast<unsigned>(std::min<int64_t>(256, (samples + 255) / 256))),
                     dim3(256), 0, s, keys, min_src, nnz, stride, band, w.cnt_mode);
  hipLaunchKernelGGL(set_mode, dim3(1), dim3(64), 0, s, w.cnt_mode, samples);
  MSREP_LAUNCHED("band_count");
  switch (value_bytes(vtype)) {
    case 8:
      return transpose_sort_t<uint64_t>(keys, min_src, static_cast<const uint64_t *>(val_src), nnz,
                                        bits, w, dminor, static_cast<uint64_t *>(dval), s, sorted);
    case 4:
      return transpose_sort_t<uint32_t>(keys, min_src, static_cast<const uint32_t *>(val_src), nnz,
                                        bits, w, dminor, static_cast<uint32_t *>(dval), s, sorted);
    default:
      return transpose_sort_t<uint16_t>(keys, min_src, static_cast<const uint16_t *>(val_src), nnz,
                                        bits, w, dminor, static_cast<uint16_t *>(dval), s, sorted);
  }
}

int key_bits(int64_t range) {
  int b = 1;
  while (b < 32 && (int64_t(1) << b) < range) ++b;
  return b;
}

msrep_status gather_entries_by(const int32_t *minor, const void *val, const int32_t *perm,
                               int64_t nnz, int32_t vtype, int32_t *dminor, void *dval,
                               hipStream_t s) {
  const int g = grid_for(nnz);
  hipLaunchKernelGGL(gather<int32_t>, dim3(g), dim3(256), 0, s, minor, perm, nnz, dminor, nullptr, 0);
  switch (value_bytes(vtype)) {
    case 8:
      hipLaunchKernelGGL(gather<uint64_t>, dim3(g), dim3(256), 0, s,
                         static_cast<const uint64_t *>(val), perm, nnz, static_cast<uint64_t *>(dval),
                         nullptr, 0);
      break;
    case 4:
      hipLaunchKernelGGL(gather<uint32_t>, dim3(g), dim3(256), 0, s,
                         static_cast<const uint32_t *>(val), perm, nnz, static_cast<uint32_t *>(dval),
                         nullptr, 0);
      break;
    default:
      hipLaunchKernelGGL(gather<uint16_t>, dim3(g), dim3(256), 0, s,
                         static_cast<const uint16_t *>(val), perm, nnz, static_cast<uint16_t *>(dval),
                         nullptr, 0);
  }
  MSREP_LAUNCHED("gather");
  return MSREP_OK;
}

}  // namespace
}  // namespace msrep

using namespace msrep;

extern "C" size_t msrep_convert_ws_bytes(const msrep_mat *src, int32_t dst_fmt) {
  if (!src || src->nnz < 0 || src->m < 0 || src->n < 0) return 0;
  const int64_t minor = std::max(src->m, src->n);
  const size_t vb = transposing(src->fmt, dst_fmt) ? value_bytes(src->vtype) : 0;
  return plan_ws(nullptr, src->nnz, minor, src->fmt == MSREP_COO_ANY, vb).bytes;
}

namespace {

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

namespace {

// COO in any order (idx: rows, idx2: columns) into any sorted format: the
// positions sorted stably by the target's minor index, then stably by its
// major index (an LSD sort on the pair), so entries equal on both keep their
// storage order.
msrep_status sort_any(const msrep_mat *src, msrep_mat *dst, Ws &w, hipStream_t s) {
  const int64_t nnz = src->nnz;
  const bool rm = row_major(dst->fmt);
  const int32_t *smaj = rm ? src->idx : src->idx2;
  const int32_t *smin = rm ? src->idx2 : src->idx;
  const int32_t maj_ext = rm ? src->m : src->n, min_ext = rm ? src->n : src->m;
  const bool dcomp = compressed(dst->fmt);
  int32_t *dptr = const_cast<int32_t *>(dst->ptr);
  if (nnz == 0) {
    if (dcomp) {
      hipLaunchKernelGGL(fill<int32_t>, dim3(grid_for(int64_t(maj_ext) + 1)), dim3(256), 0, s,
                         dptr, int64_t(maj_ext) + 1, int32_t(0));
      MSREP_LAUNCHED("fill");
    }
    return ok();
  }
  int32_t *perm = nullptr;
  uint32_t *sorted = nullptr;
  if (msrep_status st = stable_sort(smin, nnz, key_bits(min_ext), w, s, &perm, &sorted)) return st;
  MSREP_HIP(hipMemcpyAsync(w.p1, perm, 4 * static_cast<size_t>(nnz), hipMemcpyDeviceToDevice, s));
  // the major index in that order, sorted stably
  hipLaunchKernelGGL(gather<int32_t>, dim3(grid_for(nnz)), dim3(256), 0, s, smaj, w.p1, nnz,
                     w.major,
                     nullptr, 0);
  MSREP_LAUNCHED("gather");
  if (msrep_status st = stable_sort(w.major, nnz, key_bits(maj_ext), w, s, &perm, &sorted))
    return st;
  // storage positions in the final order
  hipLaunchKernelGGL(gather<int32_t>, dim3(grid_for(nnz)), dim3(256), 0, s, w.p1, perm, nnz,
                     w.major,
                     nullptr, 0);
  MSREP_LAUNCHED("gather");
  if (dcomp) {
    hipLaunchKernelGGL(rows_to_ptr, dim3(grid_for_ptr(nnz)), dim3(256), 0, s,
                       reinterpret_cast<const int32_t *>(sorted), nnz, maj_ext, dptr);
    MSREP_LAUNCHED("rows_to_ptr");
  } else {
    MSREP_HIP(hipMemcpyAsync(dst_exp(dst), sorted, 4 * static_cast<size_t>(nnz),
                             hipMemcpyDeviceToDevice, s));
  }
  if (msrep_status st = gather_entries_by(smin, src->val, w.major, nnz, src->vtype, dst_minor(dst),
                                          const_cast<void *>(dst->val), s))
    return st;
  return ok();
}

}  // namespace

extern "C" msrep_status msrep_convert(const msrep_mat *src, msrep_mat *dst, void *ws_d,
                                      size_t ws_bytes, void *stream) {
  if (msrep_status st = check_mat(src, "msrep_convert")) return st;
  if (!dst) return fail(MSREP_ERR_ARG, "msrep_convert: dst is NULL");
  if (dst->fmt < MSREP_CSR || dst->fmt > MSREP_COO_COL)
    return fail(MSREP_ERR_ARG, "msrep_convert: unknown target format %d", dst->fmt);
  if (dst->fmt == MSREP_COO_ANY)
    return fail(MSREP_ERR_UNSUPPORTED,
                "msrep_convert: COO in any order is not a target (every other format is one)");
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
  Ws w = plan_ws(ws_d, nnz, std::max(src->m, src->n), src->fmt == MSREP_COO_ANY,
                 transposing(src->fmt, dst->fmt) ? value_bytes(src->vtype) : 0);
  const size_t vb = static_cast<size_t>(value_bytes(src->vtype)) * nnz;
  int32_t *dminor = dst_minor(dst);
  if (src->fmt == MSREP_COO_ANY) return sort_any(src, dst, w, s);
  const Sides S = sides_of(src);

  if (row_major(src->fmt) == row_major(dst->fmt)) {
    // same grouping: the major index is compressed or expanded, the minor
    // index and the values are copied
    if (dcomp) {
      if (S.ptr)
        MSREP_HIP(hipMemcpyAsync(dptr, S.ptr, 4 * (static_cast<size_t>(S.major_extent) + 1),
                                 hipMemcpyDeviceToDevice, s));
      else {
        hipLaunchKernelGGL(rows_to_ptr, dim3(grid_for_ptr(nnz)), dim3(256), 0, s, S.exp, nnz,
                           S.major_extent, dptr);
        MSREP_LAUNCHED("rows_to_ptr");
      }
    } else if (nnz > 0) {
      if (S.ptr) {
        if (msrep_status st = expand(S.ptr, S.major_extent, nnz, dst_exp(dst), s))
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
    if (msrep_status st = expand(S.ptr, S.major_extent, nnz, w.major, s)) return st;
    other = w.major;
  }
  if (nnz == 0) {
    if (dcomp) {  // an empty pointer
      hipLaunchKernelGGL(fill<int32_t>, dim3(grid_for(int64_t(key_range) + 1)), dim3(256), 0, s,
                         dptr, int64_t(key_range) + 1, int32_t(0));
      MSREP_LAUNCHED("fill");
    }
    return ok();
  }
  uint32_t *sorted = nullptr;
  const int32_t band = std::max(src->m, src->n) / 64;
  if (msrep_status st = transpose_sort(key, other, src->val, src->vtype, nnz, key_bits(key_range),
                                       band, w, dminor, dval, s, &sorted))
    return st;
  if (dcomp) {
    // the pointer from the sorted keys: ptr[c] = the first position whose key
    // is >= c (each position writes the pointers of the keys it starts; no
    // atomics, so heavy columns cost nothing extra)
    hipLaunchKernelGGL(rows_to_ptr, dim3(grid_for_ptr(nnz)), dim3(256), 0, s,
                       reinterpret_cast<const int32_t *>(sorted), nnz, key_range, dptr);
    MSREP_LAUNCHED("rows_to_ptr");
  } else {
    MSREP_HIP(hipMemcpyAsync(dst_exp(dst), sorted, 4 * nnz, hipMemcpyDeviceToDevice, s));
  }
  return ok();
}
