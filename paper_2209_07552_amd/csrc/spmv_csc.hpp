// Bucketed pCSC SpMV (msRep Algorithm 5; partial vectors summed as in
// Sec. 4.3) on one GPU.
//
// Every pCSC partition contributes a partial vector over all rows, and the
// paper sums the partitions' full-length partial vectors.  On one GPU, np
// dense partial vectors would cost np*m*8 bytes, and adding each product
// straight into y with device atomics is bound by the atomic units (a few
// tens of G atomics/s, far less on power-law rows that many columns share).
// Here the partial vectors stay sparse: every product is written once,
// grouped by row bucket (2^shift consecutive rows), and each bucket is then
// summed in LDS.
//   csc_count    one workgroup (a "producer") per contiguous run of
//                partitions counts its nonzeros per bucket (LDS histogram);
//   device scan  bucket-major exclusive offsets of every producer's run;
//   csc_scatter  the producer's wavefronts walk its partitions, form the
//                products val*x[col] and write them, with the row's low
//                bits, into the producer's run of each bucket;
//   csc_plan     each bucket is cut into pieces of at most L.piece items;
//   csc_reduce   one workgroup per piece adds its products into an LDS row
//                array; a bucket of one piece writes y = alpha*sum + beta*y
//                directly, a bucket of several stores the arrays;
//   csc_merge    one thread per row of those buckets (listed by csc_plan)
//                adds the pieces' arrays in piece order.
// Streaming traffic: about (s_v + 4) + 2*(s_p + 2) + 4 bytes per nonzero
// (s_p the product size), no global atomics on y.
#pragma once

#include "scan.hpp"
#include "spmv_csr.hpp"

namespace msrep {

constexpr int kCscMinShift = 13;              // 8192-row buckets
constexpr int kCscMaxShift = 13;              // 8192 rows: 64 KB of FP64 sums
constexpr int32_t kCscMaxBuckets = 8192;      // LDS cursors of one producer
// Two resident producers per CU: the runs being written at once (producers
// x buckets lines) still mostly fit the L2, which merges the scattered
// stores into whole lines before they reach HBM.
constexpr int32_t kCscMaxProducers = 512;
constexpr int kCscScatterWaves = 16;
constexpr int64_t kCscMaxCounters = int64_t(1) << 22;
// Products summed by one workgroup: 65536 (8 per row of a bucket), or 32768
// for matrices under 2^25 nonzeros, whose few pieces otherwise leave CUs
// idle while the largest buckets' pieces finish.
constexpr int64_t kCscPiece = 65536;
constexpr int64_t kCscPieceSmall = 32768;
constexpr int64_t kCscSmallNnz = int64_t(1) << 25;
constexpr int kCscBlock = 256;                // merge blocks
constexpr int kReduceBlock = 1024;            // reduce: 64 KB of LDS rows per block
constexpr int kUnroll = 8;                    // loads in flight per thread

// Workspace carve-up of the bucketed CSC path (byte offsets).
struct CscLayout {
  int shift = 0;
  int32_t nb = 0, P = 0;
  int64_t max_pieces = 0, max_slots = 0;
  int64_t piece = 0;  // products per piece
  size_t cnt = 0, agg = 0, pbase = 0, mbase = 0, mlist = 0, prod = 0, rlo = 0, part = 0, total = 0;
};

// false when m needs more buckets than one producer's LDS holds
inline bool csc_layout(int32_t m, int64_t nnz, int32_t np, int prod_bytes, CscLayout &L) {
  int shift = kCscMinShift;
  auto buckets = [&](int s) { return (static_cast<int64_t>(m) + (int64_t(1) << s) - 1) >> s; };
  while (shift < kCscMaxShift && buckets(shift) > kCscMaxBuckets) ++shift;
  const int64_t nb = std::max<int64_t>(1, buckets(shift));
  if (nb > kCscMaxBuckets) return false;
  L.shift = shift;
  L.nb = static_cast<int32_t>(nb);
  L.P = static_cast<int32_t>(std::max<int64_t>(
      1, std::min<int64_t>({static_cast<int64_t>(std::max(np, 1)), kCscMaxProducers,
                            kCscMaxCounters / nb})));
  // sum over buckets of max(1, ceil(c/S)) < nb + nnz/S; buckets of several
  // pieces hold fewer than 2*nnz/S pieces in all
  L.piece = nnz < kCscSmallNnz ? kCscPieceSmall : kCscPiece;
  L.max_pieces = nb + nnz / L.piece + 1;
  L.max_slots = 2 * (nnz / L.piece) + 1;
  const int64_t ncnt = nb * L.P + 1;
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o += align_up(b ? b : 1, 256);
    return at;
  };
  L.cnt = take(4 * static_cast<size_t>(ncnt));
  L.agg = take(4 * static_cast<size_t>(scan::tiles(ncnt)));
  L.pbase = take(4 * static_cast<size_t>(nb + 1));
  L.mbase = take(4 * static_cast<size_t>(nb + 1));
  L.mlist = take(4 * static_cast<size_t>(nb + 1));
  // products: either one record per product (value, then a 32-bit row
  // offset) or two arrays in the same region (values, then 16-bit row
  // offsets at L.rlo); one spare slot past nnz takes the stores of masked
  // lanes
  const size_t slots = static_cast<size_t>(nnz + 1);
  L.prod = take((static_cast<size_t>(prod_bytes) + 4) * slots + 256);
  L.rlo = L.prod + align_up(static_cast<size_t>(prod_bytes) * slots, 256);
  L.part = take(8 * static_cast<size_t>(L.max_slots) << shift);
  L.total = o;
  return true;
}

template <int K>
constexpr size_t csc_lds_per_wave() {
  return align_up(kWave * K * sizeof(int32_t), 16);
}

// Product records of the packed layout: the value and the row's offset in
// its bucket, written and read with one memory instruction (12 bytes for
// FP64 values, 8 for FP32).  Scattered stores cost the memory pipeline per
// instruction and cache line, so on matrices whose rows scatter widely one
// record store beats a value store plus a 16-bit row store, at 2 more bytes.
typedef uint32_t u32x3a __attribute__((ext_vector_type(3), aligned(4)));

template <typename A>
constexpr size_t rec_bytes() {
  return sizeof(A) + 4;
}

template <typename A>
__device__ __forceinline__ void rec_store(unsigned char *__restrict__ base, int32_t at, A v,
                                          uint32_t lo) {
  unsigned char *p = base + static_cast<int64_t>(at) * static_cast<int64_t>(rec_bytes<A>());
  if constexpr (sizeof(A) == 8) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    *reinterpret_cast<u32x3a *>(p) =
        u32x3a{static_cast<uint32_t>(u), static_cast<uint32_t>(u >> 32), lo};
  } else {
    *reinterpret_cast<u32x2 *>(p) = u32x2{__builtin_bit_cast(uint32_t, v), lo};
  }
}

template <typename A>
__device__ __forceinline__ void rec_load(const unsigned char *__restrict__ base, int64_t k, A &v,
                                         uint32_t &lo) {
  const unsigned char *p = base + k * static_cast<int64_t>(rec_bytes<A>());
  if constexpr (sizeof(A) == 8) {
    const u32x3a w = __builtin_nontemporal_load(reinterpret_cast<const u32x3a *>(p));
    v = __builtin_bit_cast(A, (static_cast<uint64_t>(w.y) << 32) | w.x);
    lo = w.z;
  } else {
    const u32x2 w = __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(p));
    v = __builtin_bit_cast(A, w.x);
    lo = w.y;
  }
}

// Partitions [pa, pb) of producer p: an equal share of the np partitions.
__device__ __forceinline__ void producer_range(int p, int32_t np, int32_t P, int64_t &pa,
                                               int64_t &pb) {
  pa = static_cast<int64_t>(p) * np / P;
  pb = static_cast<int64_t>(p + 1) * np / P;
}

// cnt[t*P + p] = nonzeros of producer p whose row lies in bucket t.
// Row indices are read four per lane (16-byte loads, consecutive items), so
// a lane adds runs of equal buckets at once; the bucket of the wavefront's
// first item, which in banded matrices most lanes share, is then summed
// across the wavefront (DPP scan) and added by one lane.  The unaligned head
// and tail of the range go item by item.
__global__ __launch_bounds__(kCscScatterWaves * kWave) void csc_count(
    const int32_t *__restrict__ row_idx, int64_t nnz, const msrep_part *__restrict__ parts,
    int32_t np, int32_t P, int32_t m, int shift, int32_t nb, int32_t *__restrict__ cnt) {
  extern __shared__ int32_t hist[];
  const int p = blockIdx.x;
  const int lane = lane_id();
  for (int i = threadIdx.x; i < nb; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  int64_t pa, pb;
  producer_range(p, np, P, pa, pb);
  if (pb > pa) {
    int64_t k0 = parts[pa].start_idx, k1 = parts[pb - 1].end_idx + 1;
    k0 = k0 < 0 ? 0 : k0;
    k1 = k1 > nnz ? nnz : k1;
    k1 = k1 < k0 ? k0 : k1;
    const int64_t up4 = (k0 + 3) & ~int64_t(3), dn4 = k1 & ~int64_t(3);
    const int64_t ka = up4 < k1 ? up4 : k1;  // [k0, ka) head, [ka, kb) groups of 4
    const int64_t kb = dn4 > ka ? dn4 : ka;  // [kb, k1) tail
    auto one = [&](int64_t k) {
      const int32_t r = row_idx[k];
      if (static_cast<uint32_t>(r) < static_cast<uint32_t>(m)) atomicAdd(&hist[r >> shift], 1);
    };
    for (int64_t k = k0 + threadIdx.x; k < ka; k += blockDim.x) one(k);
    for (int64_t k = kb + threadIdx.x; k < k1; k += blockDim.x) one(k);
    const u32x4 *__restrict__ body = reinterpret_cast<const u32x4 *>(row_idx + ka);
    const int64_t ng = (kb - ka) / 4;  // groups of four items
    const int wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
    constexpr int U = 4;  // groups per lane in flight
    for (int64_t g0 = static_cast<int64_t>(wid) * kWave * U; g0 < ng;
         g0 += static_cast<int64_t>(nw) * kWave * U) {  // uniform per wavefront
      u32x4 rv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t g = g0 + u * kWave + lane;
        rv[u] = g < ng ? __builtin_nontemporal_load(body + g) : u32x4{~0u, ~0u, ~0u, ~0u};
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t r4[4] = {static_cast<int32_t>(rv[u].x), static_cast<int32_t>(rv[u].y),
                               static_cast<int32_t>(rv[u].z), static_cast<int32_t>(rv[u].w)};
        int32_t bk[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
          bk[i] = static_cast<uint32_t>(r4[i]) < static_cast<uint32_t>(m) ? (r4[i] >> shift) : -1;
        const int32_t lead = __builtin_amdgcn_readfirstlane(bk[0]);
        int32_t mine = 0;  // this lane's items in the lead bucket
        int32_t run_b = bk[0], run_n = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (bk[i] != run_b) {
            if (run_b >= 0 && run_n) {
              if (run_b == lead)
                mine += run_n;
              else
                atomicAdd(&hist[run_b], run_n);
            }
            run_b = bk[i];
            run_n = 0;
          }
          ++run_n;
        }
        if (run_b >= 0) {
          if (run_b == lead)
            mine += run_n;
          else
            atomicAdd(&hist[run_b], run_n);
        }
        // wavefront sum of the lead bucket's items
        int32_t tot = mine, none = 0;
        wave_seg_scan<int32_t>(tot, none);
        tot = __builtin_amdgcn_readlane(tot, kWave - 1);
        if (lead >= 0 && lane == 0 && tot) atomicAdd(&hist[lead], tot);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += blockDim.x) cnt[static_cast<int64_t>(i) * P + p] = hist[i];
  if (p == 0 && threadIdx.x == 0) cnt[static_cast<int64_t>(nb) * P] = 0;
}

// Local column pointer words read one chunk ahead: one 16-byte load per lane,
// 256 consecutive columns (see lp_round_load).
constexpr int kLpAhead = 4;

__device__ __forceinline__ void lp_words(rsrc_t rl, int32_t jb, int32_t (&av)[kLpAhead]) {
  lp_round_load<1>(rl, jb, av);
}

// The column of every position of a loaded chunk.  Columns that start inside
// the chunk mark their first position in the wave's LDS array (the local
// column pointer lp from j0, the column holding the chunk's first position:
// the 256 words read ahead in av0, then kLpWide words per round);
// a max-scan (DPP) carries the index forward.  ok: a position of the
// partition whose row lies in [0, m).  j0 advances to the column holding the
// next chunk's first position, taken from the lane that read the first
// column starting past the chunk (no extra load).
template <int K>
__device__ __forceinline__ void csc_columns(int32_t nloc, int32_t cb, int32_t c0, int32_t R,
                                            rsrc_t rl, int32_t m, int32_t *s_col, int32_t &j0,
                                            const int32_t (&av0)[kLpAhead],
                                            const int32_t (&rows)[K], int32_t (&col)[K],
                                            bool (&ok)[K]) {
  constexpr int CH = kWave * K;
  const int lane = lane_id();
  const int32_t ce = cb + CH < nloc ? cb + CH : nloc;
  const int32_t q0 = cb + lane * K;
#pragma unroll
  for (int t = 0; t < K; ++t) s_col[lane * K + t] = -1;
  wave_lds_sync();
  // first the 256 words read ahead, then wide rounds
  auto mark = [&](int32_t j, int32_t aw, bool in) {
    if (in && j > j0) {
      const int32_t pos = aw - cb;
      if (pos >= 0 && pos < CH) atomicMax(&s_col[pos], j);  // the non-empty column wins
    }
  };
  int32_t w0[kLpAhead];
#pragma unroll
  for (int i = 0; i < kLpAhead; ++i) w0[i] = av0[i];
  int32_t jb = j0, nxt = 0;
  int32_t tot = lp_round_scan<1>(w0, jb, R, ce, nxt, mark);
  if (tot == 4 * kWave) {
    // sparse region (runs of empty columns): wide rounds
    jb += 4 * kWave;
    for (;;) {
      tot = lp_wide_round(rl, jb, R, ce, nxt, mark);
      if (tot < kLpWide) break;
      jb += kLpWide;
    }
  }
  const int32_t j1 = jb + tot - 1;
  wave_lds_sync();
  int32_t cj[K];
  int32_t mx = j0;
#pragma unroll
  for (int t = 0; t < K; ++t) {
    const int32_t h = s_col[lane * K + t];
    mx = h > mx ? h : mx;
    cj[t] = mx;
  }
  const int32_t agg = wave_max_scan_nonneg(mx);  // values >= j0 >= 0
  int32_t cin = dpp_i<kDppWaveShr1>(agg);
  if (lane == 0) cin = j0;
#pragma unroll
  for (int t = 0; t < K; ++t) {
    const int32_t q = q0 + t;
    col[t] = c0 + (cj[t] > cin ? cj[t] : cin);
    ok[t] = q >= 0 && q < nloc && static_cast<uint32_t>(rows[t]) < static_cast<uint32_t>(m);
  }
  // the column holding the chunk's last position continues, unless it ends
  j0 = nxt > ce ? j1 : j1 + 1;
  wave_lds_sync();
}

// Partition record fields a wavefront needs (wave-uniform).
struct CscPart {
  int64_t s0;
  int32_t nloc, c0, R;
  const int32_t *lp;
};

__device__ __forceinline__ CscPart csc_part(const msrep_part *__restrict__ parts,
                                            const int32_t *__restrict__ lptr, int64_t pi) {
  const msrep_part *pp = parts + pi;
  CscPart c;
  c.s0 = uniform(pp->start_idx);
  c.nloc = static_cast<int32_t>(uniform(pp->end_idx) - c.s0 + 1);
  c.c0 = uniform(pp->start_row);
  c.R = uniform(pp->end_row) - c.c0 + 1;
  c.lp = lptr + uniform(pp->lptr_off);
  return c;
}

__device__ __forceinline__ rsrc_t lp_rsrc(const CscPart &c, bool live) {
  return make_rsrc(c.lp, live && c.R >= 0 ? static_cast<uint32_t>(c.R + 1) * 4u : 0u);
}

// LDS of one scatter producer: a cursor per bucket, a spare cursor per lane
// (masked lanes), then each wavefront's column array.
template <int K>
constexpr size_t csc_scatter_lds(int32_t nb) {
  return align_up((static_cast<size_t>(nb) + kWave) * 4, 16) + csc_lds_per_wave<K>() * kCscScatterWaves;
}

// Products of producer p go straight to their positions in its run of each
// bucket (an LDS cursor per bucket hands out positions).  Each wavefront
// walks its partitions (pa+wid, pa+wid+W, ...) as one stream of chunks.  Per
// chunk it finds the columns and issues the x gathers, then the previous
// chunk's stores and the next chunk's loads (rows, values, local column
// pointer words), and only then waits for x.  Every load is a bounds-checked
// buffer load and every lane stores (masked lanes to the spare slot at index
// nnz), so the code between the waits has no branch and the only memory
// latency left on a chunk's path is its x gather.
template <int VT, int K, bool PACK>
__global__ __launch_bounds__(kCscScatterWaves * kWave) void csc_scatter(
    const int32_t *__restrict__ row_idx, const typename vt_traits<VT>::V *__restrict__ val,
    int64_t nnz, const msrep_part *__restrict__ parts, const int32_t *__restrict__ lptr,
    int32_t np, int32_t P, const typename vt_traits<VT>::T *__restrict__ x, int32_t m, int32_t n,
    int shift, int32_t nb, const int32_t *__restrict__ off,
    typename vt_traits<VT>::A *__restrict__ prod, uint16_t *__restrict__ rlo) {
  using Tr = vt_traits<VT>;
  using V = typename Tr::V;
  using T = typename Tr::T;
  using Acc = typename Tr::A;
  constexpr int CH = kWave * K;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  int32_t *cur = reinterpret_cast<int32_t *>(lds_raw);

  const int wid = threadIdx.x / kWave;
  const int wpb = blockDim.x / kWave;
  const int lane = lane_id();
  const int p = xcd_block(blockIdx.x, gridDim.x);
  for (int i = threadIdx.x; i < nb + kWave; i += blockDim.x)
    cur[i] = i < nb ? off[static_cast<int64_t>(i) * P + p] : 0;
  __syncthreads();
  int32_t *s_col = reinterpret_cast<int32_t *>(
      lds_raw + align_up((static_cast<size_t>(nb) + kWave) * 4, 16) + wid * csc_lds_per_wave<K>());
  const uint32_t mask = (1u << shift) - 1u;
  const int32_t spare = static_cast<int32_t>(nnz);  // nnz < 2^31
  const rsrc_t rx = make_rsrc(x, static_cast<uint32_t>(n) * static_cast<uint32_t>(sizeof(T)));
  int64_t pa, pb;
  producer_range(p, np, P, pa, pb);

  // skip empty partitions: the first non-empty one at or after pi (stride wpb)
  auto first_nonempty = [&](int64_t pi, CscPart &c) {
    for (; pi < pb; pi += wpb) {
      c = csc_part(parts, lptr, pi);
      if (c.nloc > 0) break;
    }
    return pi;
  };
  CscPart cp{}, np_meta{};
  int64_t pi = first_nonempty(pa + wid, cp);
  int64_t pn = pi < pb ? first_nonempty(pi + wpb, np_meta) : pb;  // the next partition
  int32_t cb = pi < pb ? -static_cast<int32_t>(cp.s0 % K) : 0, j0 = 0;
  int32_t rows[K], av[kLpAhead];
  V v[K];
  rsrc_t rl = lp_rsrc(cp, pi < pb);
  load_items<V, K>(row_idx, val, cp.s0, cb, pi < pb ? cp.nloc : cb, rows, v);
  lp_words(rl, 0, av);
  // the previous chunk's products, positions and row bits (none yet: spare)
  Acc pr_p[K];
  int32_t at_p[K], lo_p[K];
#pragma unroll
  for (int t = 0; t < K; ++t) {
    pr_p[t] = Acc(0);
    at_p[t] = spare;
    lo_p[t] = 0;
  }
  auto store_prev = [&]() {
#pragma unroll
    for (int t = 0; t < K; ++t) {
      if constexpr (PACK) {
        rec_store<Acc>(reinterpret_cast<unsigned char *>(prod), at_p[t], pr_p[t],
                       static_cast<uint32_t>(lo_p[t]));
      } else {
        prod[at_p[t]] = pr_p[t];
        rlo[at_p[t]] = static_cast<uint16_t>(lo_p[t]);
      }
    }
  };
  while (pi < pb) {
    // ---- this chunk: columns, then the x gathers
    int32_t col[K];
    bool okk[K];
    csc_columns<K>(cp.nloc, cb, cp.c0, cp.R, rl, m, s_col, j0, av, rows, col, okk);
    T xv[K];
#pragma unroll
    for (int t = 0; t < K; ++t)
      xv[t] = buf_load<T>(rx, okk[t] && static_cast<uint32_t>(col[t]) < static_cast<uint32_t>(n)
                                  ? static_cast<uint32_t>(col[t]) * static_cast<uint32_t>(sizeof(T))
                                  : ~0u);
    store_prev();
    // ---- the next chunk (the same partition, or the first of the next
    // one); nothing is read past the last chunk
    const bool same = cb + CH < cp.nloc;
    const bool more = same || pn < pb;
    const CscPart &cq = same ? cp : np_meta;
    const int32_t cb_n = same ? cb + CH : -static_cast<int32_t>(np_meta.s0 % K);
    const int32_t j0_n = same ? j0 : 0;
    const rsrc_t rl_n = lp_rsrc(cq, more);
    int32_t rows_n[K], av_n[kLpAhead];
    V v_n[K];
    load_items<V, K>(row_idx, val, cq.s0, cb_n, more ? cq.nloc : cb_n, rows_n, v_n);
    lp_words(rl_n, j0_n, av_n);
    // ---- products and their positions in the buckets' runs
#pragma unroll
    for (int t = 0; t < K; ++t) {
      pr_p[t] = Tr::val(v[t]) * static_cast<Acc>(xv[t]);
      const int32_t slot = okk[t] ? static_cast<int32_t>(static_cast<uint32_t>(rows[t]) >> shift)
                                  : nb + lane;
      const int32_t a = atomicAdd(&cur[slot], 1);
      at_p[t] = okk[t] && static_cast<uint32_t>(a) < static_cast<uint32_t>(spare) ? a : spare;
      lo_p[t] = static_cast<int32_t>(static_cast<uint32_t>(rows[t]) & mask);
    }
    // ---- advance
    if (same) {
      cb = cb_n;
      j0 = j0_n;
    } else {
      pi = pn;
      cp = np_meta;
      cb = cb_n;
      j0 = 0;
      if (pi < pb) pn = first_nonempty(pi + wpb, np_meta);
    }
    rl = rl_n;
#pragma unroll
    for (int t = 0; t < K; ++t) {
      rows[t] = rows_n[t];
      v[t] = v_n[t];
    }
#pragma unroll
    for (int u = 0; u < kLpAhead; ++u) av[u] = av_n[u];
  }
  store_prev();
}

// The same bucketed SpMV on COO in any order (MSREP_COO_ANY): every
// partition's partial vector is kept sparse exactly as for CSC (the
// column-style merge the paper names for COO that is not row-sorted), but
// each nonzero's column is read from col_idx instead of being found from a
// local column pointer.  Partitions are equal-nnz position ranges.
template <int K>
__device__ __forceinline__ void load_cols(const int32_t *__restrict__ idx, int64_t s0, int32_t cb,
                                          int32_t nloc, int32_t (&c)[K]) {
  constexpr int CH = kWave * K;
  const int32_t span = nloc - cb < CH ? nloc - cb : CH;
  const int32_t n_ok = span > 0 ? span : 0;
  const rsrc_t ri = make_rsrc(idx + s0 + cb, static_cast<uint32_t>(n_ok) * 4u);
  const uint32_t l = static_cast<uint32_t>(lane_id() * K);
  buf_load_vec<int32_t, K, kNt>(ri, l * 4u, c);
}

template <int VT, int K, bool PACK>
__global__ __launch_bounds__(kCscScatterWaves * kWave) void coo_any_scatter(
    const int32_t *__restrict__ row_idx, const int32_t *__restrict__ col_idx,
    const typename vt_traits<VT>::V *__restrict__ val, int64_t nnz,
    const msrep_part *__restrict__ parts, int32_t np, int32_t P,
    const typename vt_traits<VT>::T *__restrict__ x, int32_t m, int32_t n, int shift, int32_t nb,
    const int32_t *__restrict__ off, typename vt_traits<VT>::A *__restrict__ prod,
    uint16_t *__restrict__ rlo) {
  using Tr = vt_traits<VT>;
  using V = typename Tr::V;
  using T = typename Tr::T;
  using Acc = typename Tr::A;
  constexpr int CH = kWave * K;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  int32_t *cur = reinterpret_cast<int32_t *>(lds_raw);
  const int wid = threadIdx.x / kWave;
  const int wpb = blockDim.x / kWave;
  const int lane = lane_id();
  const int p = xcd_block(blockIdx.x, gridDim.x);
  for (int i = threadIdx.x; i < nb + kWave; i += blockDim.x)
    cur[i] = i < nb ? off[static_cast<int64_t>(i) * P + p] : 0;
  __syncthreads();
  const uint32_t mask = (1u << shift) - 1u;
  const int32_t spare = static_cast<int32_t>(nnz);  // nnz < 2^31
  const rsrc_t rx = make_rsrc(x, static_cast<uint32_t>(n) * static_cast<uint32_t>(sizeof(T)));
  int64_t pa, pb;
  producer_range(p, np, P, pa, pb);
  // partition pi's first position and length (an empty one has none)
  auto range = [&](int64_t pi, int64_t &s0, int32_t &nloc) {
    s0 = uniform(parts[pi].start_idx);
    nloc = static_cast<int32_t>(uniform(parts[pi].end_idx) - s0 + 1);
  };
  auto first_nonempty = [&](int64_t pi, int64_t &s0, int32_t &nloc) {
    for (; pi < pb; pi += wpb) {
      range(pi, s0, nloc);
      if (nloc > 0) break;
    }
    return pi;
  };
  int64_t s_c = 0, s_n = 0;
  int32_t n_c = 0, n_n = 0;
  int64_t pi = first_nonempty(pa + wid, s_c, n_c);
  int64_t pn = pi < pb ? first_nonempty(pi + wpb, s_n, n_n) : pb;
  int32_t cb = pi < pb ? -static_cast<int32_t>(s_c % K) : 0;
  int32_t rows[K], cols[K];
  V v[K];
  load_items<V, K>(row_idx, val, s_c, cb, pi < pb ? n_c : cb, rows, v);
  load_cols<K>(col_idx, s_c, cb, pi < pb ? n_c : cb, cols);
  // the previous chunk's products, positions and row bits (none yet: spare)
  Acc pr_p[K];
  int32_t at_p[K], lo_p[K];
#pragma unroll
  for (int t = 0; t < K; ++t) {
    pr_p[t] = Acc(0);
    at_p[t] = spare;
    lo_p[t] = 0;
  }
  auto store_prev = [&]() {
#pragma unroll
    for (int t = 0; t < K; ++t) {
      if constexpr (PACK) {
        rec_store<Acc>(reinterpret_cast<unsigned char *>(prod), at_p[t], pr_p[t],
                       static_cast<uint32_t>(lo_p[t]));
      } else {
        prod[at_p[t]] = pr_p[t];
        rlo[at_p[t]] = static_cast<uint16_t>(lo_p[t]);
      }
    }
  };
  while (pi < pb) {
    bool okk[K];
    T xv[K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const int32_t q = cb + lane * K + t;
      okk[t] = q >= 0 && q < n_c && static_cast<uint32_t>(rows[t]) < static_cast<uint32_t>(m);
      xv[t] = buf_load<T>(rx, okk[t] && static_cast<uint32_t>(cols[t]) < static_cast<uint32_t>(n)
                                  ? static_cast<uint32_t>(cols[t]) * static_cast<uint32_t>(sizeof(T))
                                  : ~0u);
    }
    store_prev();
    // the next chunk (the same partition, or the first of the next one)
    const bool same = cb + CH < n_c;
    const bool more = same || pn < pb;
    const int64_t sq = same ? s_c : s_n;
    const int32_t nq = same ? n_c : n_n;
    const int32_t cb_n = same ? cb + CH : -static_cast<int32_t>(s_n % K);
    int32_t rows_n[K], cols_n[K];
    V v_n[K];
    load_items<V, K>(row_idx, val, sq, cb_n, more ? nq : cb_n, rows_n, v_n);
    load_cols<K>(col_idx, sq, cb_n, more ? nq : cb_n, cols_n);
#pragma unroll
    for (int t = 0; t < K; ++t) {
      pr_p[t] = Tr::val(v[t]) * static_cast<Acc>(xv[t]);
      const int32_t slot = okk[t] ? static_cast<int32_t>(static_cast<uint32_t>(rows[t]) >> shift)
                                  : nb + lane;
      const int32_t a = atomicAdd(&cur[slot], 1);
      at_p[t] = okk[t] && static_cast<uint32_t>(a) < static_cast<uint32_t>(spare) ? a : spare;
      lo_p[t] = static_cast<int32_t>(static_cast<uint32_t>(rows[t]) & mask);
    }
    if (same) {
      cb = cb_n;
    } else {
      pi = pn;
      s_c = s_n;
      n_c = n_n;
      cb = cb_n;
      if (pi < pb) pn = first_nonempty(pi + wpb, s_n, n_n);
    }
#pragma unroll
    for (int t = 0; t < K; ++t) {
      rows[t] = rows_n[t];
      cols[t] = cols_n[t];
      v[t] = v_n[t];
    }
  }
  store_prev();
}

// Exclusive scan of one int per thread over a block of kPlanBlock threads
// (DPP within wavefronts, wavefront totals through LDS); returns the total.
constexpr int kPlanBlock = 1024;

__device__ __forceinline__ int32_t plan_exscan(int32_t v, int32_t &excl, int32_t *sh) {
  const int lane = lane_id(), w = threadIdx.x / kWave;
  int32_t inc = v, none = 0;
  wave_seg_scan<int32_t>(inc, none);
  if (lane == kWave - 1) sh[w] = inc;
  __syncthreads();
  int32_t before = 0, total = 0;
  for (int i = 0; i < kPlanBlock / kWave; ++i) {
    before += i < w ? sh[i] : 0;
    total += sh[i];
  }
  excl = before + inc - v;
  __syncthreads();
  return total;
}

// Pieces of every bucket: pbase = exclusive scan of max(1, ceil(c_t/S)),
// mbase = exclusive scan of the piece counts of buckets with more than one
// piece (their partial-array slots); mlist = those buckets in order, their
// number in mlist[nb].  One block of kPlanBlock threads, each taking a run
// of consecutive buckets.
__global__ __launch_bounds__(kPlanBlock) void csc_plan(const int32_t *__restrict__ off, int32_t nb,
                                                       int32_t P, int64_t piece,
                                                       int32_t *__restrict__ pbase,
                                                       int32_t *__restrict__ mbase,
                                                       int32_t *__restrict__ mlist) {
  __shared__ int32_t sh[kPlanBlock / kWave];
  const int32_t per = (nb + kPlanBlock - 1) / kPlanBlock;
  const int32_t t0 = threadIdx.x * per;
  const int32_t t1 = t0 + per < nb ? t0 + per : nb;
  auto pieces = [&](int32_t t) {
    const int64_t c = static_cast<int64_t>(off[static_cast<int64_t>(t + 1) * P]) -
                      off[static_cast<int64_t>(t) * P];
    return c > 0 ? static_cast<int32_t>((c + piece - 1) / piece) : 1;
  };
  int32_t sp = 0, sm = 0, sn = 0;
  for (int32_t t = t0; t < t1; ++t) {
    const int32_t k = pieces(t);
    sp += k;
    sm += k > 1 ? k : 0;
    sn += k > 1 ? 1 : 0;
  }
  int32_t ep, em, en;
  const int32_t tp = plan_exscan(sp, ep, sh);
  const int32_t tm = plan_exscan(sm, em, sh);
  const int32_t tn = plan_exscan(sn, en, sh);
  for (int32_t t = t0; t < t1; ++t) {
    const int32_t k = pieces(t);
    pbase[t] = ep;
    mbase[t] = em;
    ep += k;
    if (k > 1) {
      em += k;
      mlist[en++] = t;
    }
  }
  if (threadIdx.x == 0) {
    pbase[nb] = tp;
    mbase[nb] = tm;
    mlist[nb] = tn;
  }
}

// One workgroup per piece (grid: an upper bound on the number of pieces).
// Offsets are clamped to nnz and partial slots to max_slots, so partition
// metadata that does not match the matrix cannot move an access outside the
// workspace.
template <typename T, typename PT, bool PACK>
__global__ __launch_bounds__(kReduceBlock) void csc_reduce(
    const PT *__restrict__ prod, const uint16_t *__restrict__ rlo, const int32_t *__restrict__ off,
    const int32_t *__restrict__ pbase, const int32_t *__restrict__ mbase, int32_t nb, int32_t P,
    int shift, int32_t m, int64_t nnz, int64_t piece, int64_t max_slots, double *__restrict__ part,
    T *__restrict__ y, double alpha, double beta) {
  extern __shared__ double acc[];
  const int32_t g = blockIdx.x;
  if (g >= pbase[nb]) return;
  int32_t lo = 0, hi = nb - 1;  // the bucket t with pbase[t] <= g < pbase[t+1]
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (pbase[mid] <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int32_t t = lo, j = g - pbase[t], npc = pbase[t + 1] - pbase[t];
  int64_t b0 = off[static_cast<int64_t>(t) * P], b1 = off[static_cast<int64_t>(t + 1) * P];
  b0 = b0 < 0 ? 0 : (b0 > nnz ? nnz : b0);
  b1 = b1 < b0 ? b0 : (b1 > nnz ? nnz : b1);
  const int64_t i0 = b0 + static_cast<int64_t>(j) * piece;
  const int64_t i1 = i0 + piece < b1 ? i0 + piece : b1;
  const int32_t span = 1 << shift;
  const uint32_t mask = static_cast<uint32_t>(span) - 1u;
  const int32_t r0 = t << shift;
  const int32_t rows = m - r0 < span ? m - r0 : span;
  for (int r = threadIdx.x; r < span; r += blockDim.x) acc[r] = 0.0;
  __syncthreads();
  // kUnroll loads in flight per thread before their LDS adds
  const int64_t bd = blockDim.x;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kUnroll * bd) {
    uint32_t rr[kUnroll];
    double pv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t k = i + u * bd;
      if constexpr (PACK) {
        PT v = PT(0);
        uint32_t lo = 0u;
        if (k < i1) rec_load<PT>(reinterpret_cast<const unsigned char *>(prod), k, v, lo);
        rr[u] = lo;
        pv[u] = static_cast<double>(v);
      } else {
        rr[u] = k < i1 ? __builtin_nontemporal_load(rlo + k) : 0u;
        pv[u] = k < i1 ? static_cast<double>(__builtin_nontemporal_load(prod + k)) : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (i + u * bd < i1) atomicAdd(&acc[rr[u] & mask], pv[u]);
  }
  __syncthreads();
  auto out = [&](int32_t r, double s) {
    const double b = beta == 0.0 ? 0.0 : beta * static_cast<double>(y[r0 + r]);
    y[r0 + r] = static_cast<T>(alpha * s + b);
  };
  if (npc == 1) {
    for (int r = threadIdx.x; r < rows; r += blockDim.x) out(r, acc[r]);
    return;
  }
  if (mbase[t] < 0 || static_cast<int64_t>(mbase[t]) + npc > max_slots) return;
  double *mine = part + (static_cast<int64_t>(mbase[t] + j) << shift);
  for (int r = threadIdx.x; r < rows; r += blockDim.x) mine[r] = acc[r];
}

// Rows of buckets cut into several pieces: the pieces' arrays added in piece
// order, one thread per row.  Only the mlist[nb] buckets listed by csc_plan
// have rows here; the blocks stride over (listed bucket, 256-row block).
template <typename T>
__global__ __launch_bounds__(kCscBlock) void csc_merge(const int32_t *__restrict__ pbase,
                                                      const int32_t *__restrict__ mbase,
                                                      const int32_t *__restrict__ mlist,
                                                      int32_t nb, int shift, int32_t m,
                                                      int64_t max_slots,
                                                      const double *__restrict__ part,
                                                      T *__restrict__ y, double alpha,
                                                      double beta) {
  const int32_t nlist = mlist[nb];
  const int32_t rb = (1 << shift) / kCscBlock;  // row blocks per bucket
  for (int64_t w = blockIdx.x; w < static_cast<int64_t>(nlist) * rb; w += gridDim.x) {
    const int32_t t = mlist[w / rb];
    const int32_t npc = pbase[t + 1] - pbase[t];
    if (npc <= 1 || mbase[t] < 0 || static_cast<int64_t>(mbase[t]) + npc > max_slots) continue;
    const int32_t r = static_cast<int32_t>(w % rb) * kCscBlock + threadIdx.x;
    const int32_t r0 = t << shift;
    if (r0 + r >= m) continue;
    const double *base = part + (static_cast<int64_t>(mbase[t]) << shift) + r;
    double s = 0.0;
    int32_t q = 0;
    for (; q + kUnroll <= npc; q += kUnroll) {
      double v[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) v[u] = base[static_cast<int64_t>(q + u) << shift];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) s += v[u];
    }
    for (; q < npc; ++q) s += base[static_cast<int64_t>(q) << shift];
    const double b = beta == 0.0 ? 0.0 : beta * static_cast<double>(y[r0 + r]);
    y[r0 + r] = static_cast<T>(alpha * s + b);
  }
}

}  // namespace msrep
