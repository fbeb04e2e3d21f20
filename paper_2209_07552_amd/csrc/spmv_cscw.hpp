// Windowed pCSC SpMV (msRep Algorithm 5, partial vectors summed as in
// Sec. 4.3) for matrices whose partitions touch few row ranges: banded and
// stencil matrices, where the columns of a run of partitions reach a handful
// of narrow row bands.
//
// The bucketed path (spmv_csc.hpp) writes every product to HBM and reads it
// back; here the partial vector of a producer (a workgroup owning a run of
// consecutive partitions) is accumulated in LDS instead, over the row
// windows (256 consecutive rows each) that its nonzeros touch, and only
// those windows' sums are written: one FP64 per row of each window, a few
// per row of the matrix for a 7-point stencil instead of one product per
// nonzero.  A window is then completed by adding, in one pass, the slices
// every producer wrote for it (the column merge of Sec. 4.3 over the
// producers' partial vectors, kept as windows rather than full length).
//
//   cscw_windows   (structure) per producer: the windows its rows touch, as
//                  an LDS bitmap over the kWinMap windows from its first;
//                  the first kWinMax present windows are the producer's LDS
//                  windows; any row outside them marks the matrix "spilled";
//                  every listed window counts one contributor;
//   device scan    contributor offsets per window;
//   cscw_inv_fill  (structure) the contributor lists of every window;
//   cscw_zero      (numeric) clears the spill accumulator, only if spilled;
//   cscw_tile      (numeric) per producer: products val*x[col] added into
//                  its LDS windows (ds_add_f64), a row outside them into the
//                  spill accumulator with a device atomic; then the windows
//                  are written out;
//   cscw_merge     (numeric) per window: y = alpha*(sum of its slices
//                  [+ spill accumulator]) + beta*y.
// Any matrix is computed correctly; matrices whose producers touch more than
// kWinMax windows (power-law rows everywhere) pay device atomics for the
// rest, which the autotuner avoids by keeping the bucketed path.
#pragma once

#include "spmv_csc.hpp"

namespace msrep {

constexpr int kWinShift = 8;                  // 256-row windows
constexpr int kWinRows = 1 << kWinShift;
constexpr int kWinMax = 30;                   // LDS windows per producer (60 KB of FP64)
constexpr int kWinMap = 2048;                 // windows a producer's map spans
constexpr int kWinWaves = 8;                  // wavefronts per producer (two producers per CU)
constexpr int64_t kWinProducerNnz = 12288;    // nonzeros per producer (1.75k stencil columns: 26 windows)
constexpr int kWinMergeBlock = 256;           // one row per thread

// Workspace of the windowed path: structure regions (absolute offsets, after
// everything else) and numeric regions (relative to the bucketed products).
struct CscwLayout {
  int32_t P = 0;        // producers
  int64_t nwin = 0;     // windows of m
  // structure
  size_t wlist = 0, wcnt = 0, flags = 0, inv_cnt = 0, inv_off = 0, inv_agg = 0, inv_list = 0;
  size_t struct_end = 0;
  // numeric (relative to the numeric base)
  size_t part = 0, yacc = 0, numeric_bytes = 0;
};

inline int32_t cscw_producers(int64_t nnz, int32_t np) {
  const int64_t want = (nnz + kWinProducerNnz - 1) / kWinProducerNnz;
  return static_cast<int32_t>(std::max<int64_t>(1, std::min<int64_t>(want, std::max(np, 1))));
}

// Placement in the CSC workspace of L (the bucketed layout): the numeric
// regions (window slices, spill sums) start at L.prod and may overlap only
// the bucketed numeric regions (one path runs per call); the structure
// regions follow both, so that neither path's numeric kernels can reach
// either path's structure.  The workspace ends at struct_end.
inline void cscw_layout(int32_t m, int64_t nnz, int32_t np, const CscLayout &L, CscwLayout &W) {
  W.P = cscw_producers(nnz, np);
  W.nwin = (static_cast<int64_t>(m) + kWinRows - 1) >> kWinShift;
  const size_t pairs = static_cast<size_t>(W.P) * kWinMax;
  size_t q = 0;
  auto takeq = [&](size_t b) {
    const size_t at = q;
    q += align_up(b ? b : 1, 256);
    return at;
  };
  W.part = takeq(8 * pairs * kWinRows);
  W.yacc = takeq(8 * static_cast<size_t>(m));
  W.numeric_bytes = q;
  size_t o = std::max(L.total, L.prod + W.numeric_bytes);
  auto take = [&](size_t b) {
    const size_t at = o;
    o += align_up(b ? b : 1, 256);
    return at;
  };
  W.wlist = take(4 * pairs);
  W.wcnt = take(4 * static_cast<size_t>(W.P));
  W.flags = take(16);  // [0]: spilled
  W.inv_cnt = take(4 * static_cast<size_t>(W.nwin + 1));
  W.inv_off = take(4 * static_cast<size_t>(W.nwin + 1));
  W.inv_agg = take(4 * static_cast<size_t>(scan::tiles(W.nwin + 1) + 1));
  W.inv_list = take(4 * pairs);
  W.struct_end = o;
}

__global__ void cscw_fill_i32(int32_t *__restrict__ a, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    a[i] = v;
}

// The windows of producer p: the first present window w0 (a block min over
// its rows), an LDS bitmap of the kWinMap windows from w0, the first kWinMax
// present ones listed in order.  Rows past the map, or present windows past
// the first kWinMax, spill.
__global__ __launch_bounds__(1024) void cscw_windows(
    const int32_t *__restrict__ row_idx, int64_t nnz, const msrep_part *__restrict__ parts,
    int32_t np, int32_t P, int32_t m, int32_t *__restrict__ wlist, int32_t *__restrict__ wcnt,
    int32_t *__restrict__ flags, int32_t *__restrict__ inv_cnt) {
  __shared__ uint32_t bits[kWinMap / 32];
  __shared__ int32_t s_min, s_spill, s_cnt;
  const int p = blockIdx.x;
  for (int i = threadIdx.x; i < kWinMap / 32; i += blockDim.x) bits[i] = 0u;
  if (threadIdx.x == 0) {
    s_min = 0x7fffffff;
    s_spill = 0;
    s_cnt = 0;
  }
  __syncthreads();
  int64_t pa, pb;
  producer_range(p, np, P, pa, pb);
  int64_t k0 = 0, k1 = 0;
  if (pb > pa) {
    k0 = parts[pa].start_idx;
    k1 = parts[pb - 1].end_idx + 1;
    k0 = k0 < 0 ? 0 : k0;
    k1 = k1 > nnz ? nnz : k1;
    k1 = k1 < k0 ? k0 : k1;
  }
  int32_t mn = 0x7fffffff;
  for (int64_t k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
    const int32_t r = row_idx[k];
    if (static_cast<uint32_t>(r) < static_cast<uint32_t>(m)) mn = r < mn ? r : mn;
  }
  atomicMin(&s_min, mn);
  __syncthreads();
  const int32_t w0 = s_min == 0x7fffffff ? 0 : (s_min >> kWinShift);
  bool spill = false;
  for (int64_t k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
    const int32_t r = row_idx[k];
    if (static_cast<uint32_t>(r) >= static_cast<uint32_t>(m)) continue;
    const int32_t d = (r >> kWinShift) - w0;
    if (d < kWinMap)
      atomicOr(&bits[d >> 5], 1u << (d & 31));
    else
      spill = true;
  }
  if (spill) s_spill = 1;
  __syncthreads();
  if (threadIdx.x < kWave) {
    // list the present windows in order, kWinMax at most (one wavefront)
    const int lane = threadIdx.x;
    int32_t base = 0;
    for (int b0 = 0; b0 < kWinMap / 32; b0 += kWave) {
      const uint32_t w = b0 + lane < kWinMap / 32 ? bits[b0 + lane] : 0u;
      const int32_t c = __popc(w);
      int32_t incl = c, none = 0;
      wave_seg_scan<int32_t>(incl, none);
      int32_t at = base + incl - c;
      uint32_t rest = w;
      while (rest) {
        const int bit = __ffs(rest) - 1;
        rest &= rest - 1;
        if (at < kWinMax) {
          const int32_t win = w0 + (b0 + lane) * 32 + bit;
          wlist[static_cast<int64_t>(p) * kWinMax + at] = win;
          atomicAdd(&inv_cnt[win], 1);
        }
        ++at;
      }
      base += __builtin_amdgcn_readlane(incl, kWave - 1);
    }
    if (lane == 0) {
      wcnt[p] = base < kWinMax ? base : kWinMax;
      if (base > kWinMax || s_spill) atomicOr(&flags[0], 1);
    }
  }
}

// Contributor lists: window w's entries inv_list[inv_off[w] ..
// inv_off[w+1]) name the (producer, slot) pairs p*kWinMax + i that cover it.
// inv_cnt counts down to zero as positions are handed out.
__global__ void cscw_inv_fill(const int32_t *__restrict__ wlist, const int32_t *__restrict__ wcnt,
                              int32_t P, const int32_t *__restrict__ inv_off,
                              int32_t *__restrict__ inv_cnt, int32_t *__restrict__ inv_list) {
  const int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  const int32_t p = static_cast<int32_t>(g / kWinMax), i = static_cast<int32_t>(g % kWinMax);
  if (p >= P || i >= wcnt[p]) return;
  const int32_t w = wlist[g];
  const int32_t pos = inv_off[w] + atomicSub(&inv_cnt[w], 1) - 1;
  inv_list[pos] = static_cast<int32_t>(g);
}

__global__ void cscw_zero(const int32_t *__restrict__ flags, double *__restrict__ yacc, int64_t m) {
  if (!flags[0]) return;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < m;
       i += int64_t(gridDim.x) * blockDim.x)
    yacc[i] = 0.0;
}

// LDS of one tile producer: the window sums, the direct map from window
// offset to LDS slot, each wavefront's column array (CSC).
template <int K>
constexpr size_t cscw_lds() {
  return align_up(8 * static_cast<size_t>(kWinMax) * kWinRows, 16) + align_up(kWinMap, 16) +
         csc_lds_per_wave<K>() * kWinWaves;
}

// Producer p's products into its LDS windows.  COLS: columns read from
// col_idx (COO sorted by column or in any order); otherwise from the local
// column pointer (CSC).
template <int VT, int K, bool COLS>
__global__ __launch_bounds__(kWinWaves * kWave) void cscw_tile(
    const int32_t *__restrict__ row_idx, const int32_t *__restrict__ col_idx,
    const typename vt_traits<VT>::V *__restrict__ val, const msrep_part *__restrict__ parts,
    const int32_t *__restrict__ lptr, int32_t np, int32_t P,
    const typename vt_traits<VT>::T *__restrict__ x, int32_t m, int32_t n,
    const int32_t *__restrict__ wlist, const int32_t *__restrict__ wcnt,
    double *__restrict__ part, double *__restrict__ yacc) {
  using Tr = vt_traits<VT>;
  using V = typename Tr::V;
  using T = typename Tr::T;
  constexpr int CH = kWave * K;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double *acc = reinterpret_cast<double *>(lds_raw);
  int8_t *dmap = reinterpret_cast<int8_t *>(lds_raw + align_up(8 * static_cast<size_t>(kWinMax) * kWinRows, 16));
  const int wid = threadIdx.x / kWave;
  const int wpb = blockDim.x / kWave;
  const int p = xcd_block(blockIdx.x, gridDim.x);
  int32_t *s_col = reinterpret_cast<int32_t *>(
      lds_raw + align_up(8 * static_cast<size_t>(kWinMax) * kWinRows, 16) + align_up(kWinMap, 16) +
      wid * csc_lds_per_wave<K>());
  const int32_t nw = wcnt[p];
  const int32_t w0 = nw > 0 ? wlist[static_cast<int64_t>(p) * kWinMax] : 0;
  for (int i = threadIdx.x; i < kWinMap; i += blockDim.x) dmap[i] = -1;
  for (int i = threadIdx.x; i < nw * kWinRows; i += blockDim.x) acc[i] = 0.0;
  __syncthreads();
  if (threadIdx.x < nw) dmap[wlist[static_cast<int64_t>(p) * kWinMax + threadIdx.x] - w0] =
      static_cast<int8_t>(threadIdx.x);
  __syncthreads();
  const rsrc_t rx = make_rsrc(x, static_cast<uint32_t>(n) * static_cast<uint32_t>(sizeof(T)));
  int64_t pa, pb;
  producer_range(p, np, P, pa, pb);
  auto part_of = [&](int64_t pi, CscPart &c) {
    if constexpr (COLS) {
      c.s0 = uniform(parts[pi].start_idx);
      c.nloc = static_cast<int32_t>(uniform(parts[pi].end_idx) - c.s0 + 1);
      c.c0 = 0;
      c.R = 0;
      c.lp = nullptr;
    } else {
      c = csc_part(parts, lptr, pi);
    }
  };
  // A position in the wavefront's stream of chunks: partition pi (pb when
  // the stream is over), its record, the chunk's first local position and,
  // for CSC, the local column holding it.
  struct Cur {
    int64_t pi;
    CscPart c;
    int32_t cb, j0;
  };
  auto first_at = [&](int64_t pi, Cur &u) {
    u.c = CscPart{};  // a finished stream reads nothing (empty resources)
    for (; pi < pb; pi += wpb) {
      part_of(pi, u.c);
      if (u.c.nloc > 0) break;
    }
    if (pi >= pb) u.c = CscPart{};
    u.pi = pi;
    u.cb = pi < pb ? -static_cast<int32_t>(u.c.s0 % K) : 0;
    u.j0 = 0;
  };
  // the chunk after u (j0 is the column csc_columns left for it)
  auto next_of = [&](const Cur &u, Cur &v) {
    if (u.pi < pb && u.cb + CH < u.c.nloc) {
      v = u;
      v.cb = u.cb + CH;
    } else {
      first_at(u.pi < pb ? u.pi + wpb : pb, v);
    }
  };
  auto load_chunk = [&](const Cur &u, int32_t (&r)[K], V (&vv)[K], int32_t (&cc)[K],
                        int32_t (&aw)[kLpAhead], rsrc_t &rl) {
    const bool live = u.pi < pb;
    load_items<V, K>(row_idx, val, u.c.s0, u.cb, live ? u.c.nloc : u.cb, r, vv);
    if constexpr (COLS) {
      load_cols<K>(col_idx, u.c.s0, u.cb, live ? u.c.nloc : u.cb, cc);
    } else {
      rl = lp_rsrc(u.c, live);
      lp_words(rl, u.j0, aw);
    }
  };
  // columns (and which positions count) of a loaded chunk; for CSC this
  // advances u.j0 to the column that continues into the next chunk
  auto columns = [&](Cur &u, const int32_t (&r)[K], const int32_t (&cc)[K],
                     const int32_t (&aw)[kLpAhead], rsrc_t rl, int32_t (&col)[K], bool (&okk)[K]) {
    if constexpr (COLS) {
      const int32_t q0 = u.cb + lane_id() * K;
#pragma unroll
      for (int t = 0; t < K; ++t) {
        col[t] = cc[t];
        okk[t] = u.pi < pb && q0 + t >= 0 && q0 + t < u.c.nloc &&
                 static_cast<uint32_t>(r[t]) < static_cast<uint32_t>(m);
      }
    } else {
      csc_columns<K>(u.pi < pb ? u.c.nloc : 0, u.cb, u.c.c0, u.c.R, rl, m, s_col, u.j0, aw, r,
                     col, okk);
    }
  };
  auto gather = [&](const int32_t (&col)[K], const bool (&okk)[K], T (&xv)[K]) {
#pragma unroll
    for (int t = 0; t < K; ++t)
      xv[t] = buf_load<T>(rx, okk[t] && static_cast<uint32_t>(col[t]) < static_cast<uint32_t>(n)
                                  ? static_cast<uint32_t>(col[t]) * static_cast<uint32_t>(sizeof(T))
                                  : ~0u);
  };
  // Software pipeline over the wavefront's chunks: entering an iteration,
  // chunk a has its x gather in flight and chunk b (the next) its loads;
  // the iteration works out b's columns and issues b's gather and the loads
  // of the chunk after b, and only then forms a's products, so each x gather
  // has a whole iteration to arrive.
  Cur ua, ub;
  first_at(pa + wid, ua);
  int32_t ra[K], ca[K], aa[kLpAhead], rb[K], cbv[K], ab[kLpAhead];
  V va[K], vb[K];
  rsrc_t rla, rlb;
  load_chunk(ua, ra, va, ca, aa, rla);
  int32_t cola[K];
  bool oka[K];
  columns(ua, ra, ca, aa, rla, cola, oka);
  T xa[K];
  gather(cola, oka, xa);
  next_of(ua, ub);
  load_chunk(ub, rb, vb, cbv, ab, rlb);
  while (ua.pi < pb) {
    // ---- chunk b: columns, x gather; the chunk after it: loads
    int32_t colb[K];
    bool okb[K];
    columns(ub, rb, cbv, ab, rlb, colb, okb);
    T xb[K];
    gather(colb, okb, xb);
    Cur uc;
    next_of(ub, uc);
    int32_t rc[K], ccv[K], ac[kLpAhead];
    V vc[K];
    rsrc_t rlc;
    load_chunk(uc, rc, vc, ccv, ac, rlc);
    // ---- chunk a: products into the windows (FP64 sums)
#pragma unroll
    for (int t = 0; t < K; ++t) {
      if (!oka[t]) continue;
      const double pr = static_cast<double>(Tr::val(va[t]) * static_cast<typename Tr::A>(xa[t]));
      const int32_t d = (ra[t] >> kWinShift) - w0;
      const int32_t slot = static_cast<uint32_t>(d) < static_cast<uint32_t>(kWinMap) ? dmap[d] : -1;
      if (slot >= 0)
        atomicAdd(&acc[slot * kWinRows + (ra[t] & (kWinRows - 1))], pr);
      else
        atomicAdd(&yacc[ra[t]], pr);
    }
    // ---- rotate
    ua = ub;
    ub = uc;
#pragma unroll
    for (int t = 0; t < K; ++t) {
      ra[t] = rb[t];
      va[t] = vb[t];
      oka[t] = okb[t];
      xa[t] = xb[t];
      rb[t] = rc[t];
      vb[t] = vc[t];
      if constexpr (COLS) cbv[t] = ccv[t];
    }
    if constexpr (!COLS) {
#pragma unroll
      for (int u = 0; u < kLpAhead; ++u) ab[u] = ac[u];
    }
    rlb = rlc;
  }
  __syncthreads();
  // the windows out, coalesced
  double *dst = part + static_cast<int64_t>(p) * kWinMax * kWinRows;
  for (int i = threadIdx.x; i < nw * kWinRows; i += blockDim.x) dst[i] = acc[i];
}

// Window w: y = alpha * (its producers' slices [+ the spill sums]) + beta*y.
// The slices are read four at a time, so each thread keeps eight loads in
// flight.
template <typename T, bool BETA0>
__global__ __launch_bounds__(kWinMergeBlock) void cscw_merge(
    const int32_t *__restrict__ inv_off, const int32_t *__restrict__ inv_list,
    const int32_t *__restrict__ flags, const double *__restrict__ part,
    const double *__restrict__ yacc, int32_t m, T *__restrict__ y, double alpha, double beta) {
  const int64_t w = blockIdx.x;
  const int32_t a = inv_off[w], b = inv_off[w + 1];
  const bool spilled = flags[0] != 0;
  constexpr int R = kWinRows / kWinMergeBlock;
  constexpr int U = 4;
  double s[R];
#pragma unroll
  for (int r = 0; r < R; ++r) s[r] = 0.0;
  for (int32_t j = a; j < b; j += U) {
    double v[U][R];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t jj = j + u < b ? j + u : a;  // (re-reads a slice, added as 0)
      const double *src = part + static_cast<int64_t>(inv_list[jj]) * kWinRows;
#pragma unroll
      for (int r = 0; r < R; ++r) v[u][r] = src[threadIdx.x + r * kWinMergeBlock];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int r = 0; r < R; ++r) s[r] += j + u < b ? v[u][r] : 0.0;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t row = (w << kWinShift) + threadIdx.x + r * kWinMergeBlock;
    if (row >= m) continue;
    double v = s[r];
    if (spilled) v += yacc[row];
    y[row] = static_cast<T>(BETA0 ? alpha * v : alpha * v + beta * static_cast<double>(y[row]));
  }
}

}  // namespace msrep
