// Wave-per-partition CSR SpMV (pCSR, msRep Algorithm 3) for CDNA wave64.
//
// Each wavefront owns one equal-nnz partition and streams its nonzeros in
// chunks of 64*K (K per lane, thread-contiguous, vector loads aligned to K).
// For every chunk:
//   1. products val*x[col] in registers;
//   2. rows of the chunk come from the partition's local pointer: every row
//      that starts inside the chunk marks its first position in a per-wave
//      LDS byte array (head flags);
//   3. a segmented inclusive scan of the products (sequential over the K
//      items of a lane, then a 6-step Hillis-Steele scan across lanes) is
//      stored in LDS, so a row's in-chunk sum is the scan value at its last
//      position;
//   4. lanes take rows and write y coalesced; the row still open at the end
//      of the chunk is carried (in FP64 for FP32 values) into the next chunk.
// Rows wholly inside the partition are written directly.  The partition's
// first row when start_flag is set (head) and its last row when end_flag is
// set (tail) are partial: their sums go to the carry buffer and the boundary
// merge kernel completes them.  Empty rows between this partition and the
// next one (and, for the first partition, before it) get beta*y here.
#pragma once

#include "common.hpp"

namespace msrep {

template <int VT>
struct vt_traits;
template <>
struct vt_traits<MSREP_F64> {
  using V = double;  // stored value
  using T = double;  // x, y
  using A = double;  // in-chunk accumulation
  __device__ static A val(V v) { return v; }
};
template <>
struct vt_traits<MSREP_F32> {
  using V = float;
  using T = float;
  using A = float;
  __device__ static A val(V v) { return v; }
};
template <>
struct vt_traits<MSREP_BF16> {
  using V = uint16_t;
  using T = float;
  using A = float;
  __device__ static A val(V v) { return bf16_to_f32(v); }
};

// Load K consecutive items starting at an index that is a multiple of K.
template <typename E, int K>
__device__ __forceinline__ void load_vec(const E *__restrict__ p, E (&out)[K]) {
  constexpr int bytes = K * sizeof(E);
  static_assert(bytes % 4 == 0, "vector of whole dwords");
  if constexpr (bytes % 16 == 0) {
    const u32x4 *q = reinterpret_cast<const u32x4 *>(p);
#pragma unroll
    for (int v = 0; v < bytes / 16; ++v) {
      const u32x4 w = __builtin_nontemporal_load(q + v);
      uint32_t *o = reinterpret_cast<uint32_t *>(out) + 4 * v;
      o[0] = w.x;
      o[1] = w.y;
      o[2] = w.z;
      o[3] = w.w;
    }
  } else if constexpr (bytes == 8) {
    const u32x2 w = __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(p));
    uint32_t *o = reinterpret_cast<uint32_t *>(out);
    o[0] = w.x;
    o[1] = w.y;
  } else {
#pragma unroll
    for (int t = 0; t < K; ++t) out[t] = p[t];
  }
}

// The K items of a lane at local positions q0 .. q0+K-1 of the chunk that
// starts at local position cb of a partition whose first nonzero is s0 and
// which holds nloc nonzeros.  The buffer resources cover exactly the chunk's
// positions inside the partition, so items past its end read as 0; items
// before the partition start (q < 0) are masked to index -1 and value 0.
template <typename V, int K>
__device__ __forceinline__ void load_items(const int32_t *__restrict__ idx,
                                           const V *__restrict__ val, int64_t s0, int32_t cb,
                                           int32_t nloc, int32_t (&c)[K], V (&v)[K]) {
  constexpr int CH = kWave * K;
  const int32_t span = nloc - cb < CH ? nloc - cb : CH;  // positions cb .. cb+span-1 exist
  const int32_t n_ok = span > 0 ? span : 0;
  const rsrc_t ri = make_rsrc(idx + s0 + cb, static_cast<uint32_t>(n_ok) * 4u);
  const uint32_t l = static_cast<uint32_t>(lane_id() * K);
  buf_load_vec<int32_t, K, kNt>(ri, l * 4u, c);
  if constexpr (sizeof(V) >= 4) {
    const rsrc_t rv = make_rsrc(val + s0 + cb, static_cast<uint32_t>(n_ok) * sizeof(V));
    buf_load_vec<V, K, kNt>(rv, l * static_cast<uint32_t>(sizeof(V)), v);
  } else {
    // the hardware bounds check is per dword: cover whole dwords only and
    // fetch an odd last element with a 16-bit load of its own
    const rsrc_t rv = make_rsrc(val + s0 + cb, (static_cast<uint32_t>(n_ok) * 2u) & ~3u);
    buf_load_vec<V, K, kNt>(rv, l * 2u, v);
    const uint32_t last = static_cast<uint32_t>(n_ok - 1);
    const rsrc_t rt = make_rsrc(val + s0 + cb + (n_ok > 0 ? n_ok - 1 : 0), (n_ok & 1) ? 2u : 0u);
    const uint32_t tt = last - l;  // item of this lane that is the odd tail, if < K
    const V tail = buf_load<V>(rt, tt < static_cast<uint32_t>(K) ? 0u : 4u);
#pragma unroll
    for (int t = 0; t < K; ++t) v[t] = (n_ok & 1) && tt == static_cast<uint32_t>(t) ? tail : v[t];
  }
#pragma unroll
  for (int t = 0; t < K; ++t) {
    const int32_t q = cb + static_cast<int32_t>(l) + t;
    const bool in = q >= 0 && q < nloc;
    c[t] = in ? c[t] : -1;
    v[t] = in ? v[t] : V(0);
  }
}

// Rows covering at most this many positions of a chunk are summed by one
// lane each; a chunk holding a longer row uses the segmented scan.
constexpr int kShortRow = 32;

// One round over the local pointer words of kLpWide consecutive rows (CSR)
// or columns (CSC) from jb: lane L holds jb + 256*i + 4*L + e (kLpWideLoads
// 16-byte loads), words past R read as INT_MAX.  visit(j, word, in) sees every word;
// in = j <= R-1 and the word lies before ce.  Returns how many are in (a
// prefix, the pointer being non-decreasing) and, when that is below
// kLpWide, sets nxt to the word just past them.  Chunks over runs of empty
// rows or columns span thousands of them; this reads them in few dependent
// rounds.
constexpr int kLpWideLoads = 2;
constexpr int kLpWide = kLpWideLoads * 4 * kWave;

// The words of a round of L 16-byte loads per lane from jb (lane L holds
// jb + 256*i + 4*L + e).
template <int L>
__device__ __forceinline__ void lp_round_load(rsrc_t rl, int32_t jb, int32_t (&w)[4 * L]) {
  const int lane = lane_id();
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(
        rl, static_cast<uint32_t>(jb + i * 4 * kWave + 4 * lane) * 4u, 0, 0);
    w[4 * i] = static_cast<int32_t>(q.x);
    w[4 * i + 1] = static_cast<int32_t>(q.y);
    w[4 * i + 2] = static_cast<int32_t>(q.z);
    w[4 * i + 3] = static_cast<int32_t>(q.w);
  }
}

// Scan of a loaded round (see lp_wide_round).
template <int L, typename F>
__device__ __forceinline__ int32_t lp_round_scan(int32_t (&w)[4 * L], int32_t jb, int32_t R,
                                                 int32_t ce, int32_t &nxt, F &&visit) {
  const int lane = lane_id();
  int32_t tot = 0;
#pragma unroll
  for (int i = 0; i < L; ++i) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int32_t j = jb + i * 4 * kWave + 4 * lane + e;
      const int32_t aw = j <= R ? w[4 * i + e] : 0x7fffffff;
      w[4 * i + e] = aw;
      const bool in = j <= R - 1 && aw < ce;
      visit(j, aw, in);
      tot += __popcll(__ballot(in));
    }
  }
  if (tot < L * 4 * kWave) {
    // the word of row jb + tot: load tot / 256, lane (tot % 256) / 4, element tot % 4
    const int i_sel = tot / (4 * kWave), e_sel = tot % 4;
    int32_t pick = 0;
#pragma unroll
    for (int i = 0; i < L; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (i == i_sel && e == e_sel) pick = w[4 * i + e];
    nxt = __builtin_amdgcn_readlane(pick, (tot % (4 * kWave)) / 4);
  }
  return tot;
}

template <int L = kLpWideLoads, typename F>
__device__ __forceinline__ int32_t lp_wide_round(rsrc_t rl, int32_t jb, int32_t R, int32_t ce,
                                                 int32_t &nxt, F &&visit) {
  int32_t w[4 * L];
  lp_round_load<L>(rl, jb, w);
  return lp_round_scan<L>(w, jb, R, ce, nxt, static_cast<F &&>(visit));
}

// Rows handled per round of the loops over many rows of one chunk (loads in
// flight per lane).  The register-lean CSR variant (one chunk loaded ahead,
// also the batched kernel's) takes one batch and one-load rounds, keeping
// its occupancy.
constexpr int kRowBatch = 4;

// Per-wave LDS footprint of the CSR/COO kernels.
template <int VT, int K>
constexpr size_t seg_lds_per_wave() {
  return align_up(kWave * K * sizeof(typename vt_traits<VT>::A), 16) + align_up(kWave * K, 16);
}

template <typename T>
__device__ __forceinline__ void store_y(T *__restrict__ y, int32_t r, double v, double alpha,
                                       double beta, bool beta0) {
  const double out = beta0 ? alpha * v : alpha * v + beta * static_cast<double>(y[r]);
  y[r] = static_cast<T>(out);
}

// Rows [lo, hi) get y = beta*y (0 when beta == 0), lanes striding.
template <typename T>
__device__ __forceinline__ void scale_rows(T *__restrict__ y, int32_t lo, int32_t hi, double beta,
                                           bool beta0) {
  for (int32_t r = lo + lane_id(); r < hi; r += kWave)
    y[r] = beta0 ? static_cast<T>(0) : static_cast<T>(beta * static_cast<double>(y[r]));
}

// One wavefront processes partition p of a CSR matrix (the routine shared by
// the single-matrix kernel and the persistent batched kernel).  `carry`
// points at this matrix's two FP64 slots per partition; `my` at this
// wavefront's LDS region (seg_lds_per_wave bytes).
template <int VT, int K, bool BETA0, int PF = 1>
__device__ __forceinline__ void csr_partition(
    const int32_t *__restrict__ col, const typename vt_traits<VT>::V *__restrict__ val,
    const msrep_part *__restrict__ parts, const int32_t *__restrict__ lptr, int32_t np, int32_t p,
    const typename vt_traits<VT>::T *__restrict__ x, typename vt_traits<VT>::T *__restrict__ y,
    int32_t m, int32_t n, double alpha, double beta, double *__restrict__ carry,
    unsigned char *my) {
  using Tr = vt_traits<VT>;
  using V = typename Tr::V;
  using T = typename Tr::T;
  using Acc = typename Tr::A;
  constexpr int CH = kWave * K;
  constexpr int RB = PF == 2 ? kRowBatch : 1;      // see kRowBatch
  constexpr int WL = PF == 2 ? kLpWideLoads : 1;
  const int lane = lane_id();
  Acc *s_sum = reinterpret_cast<Acc *>(my);
  unsigned char *s_head = my + align_up(CH * sizeof(Acc), 16);

  const msrep_part *pp = parts + p;
  const int64_t s0 = uniform(pp->start_idx);
  const int64_t e0 = uniform(pp->end_idx);
  const int32_t r0 = uniform(pp->start_row);
  const int32_t R = uniform(pp->end_row) - r0 + 1;
  const int32_t sflag = uniform(pp->start_flag);
  const int32_t eflag = uniform(pp->end_flag);
  const int32_t *__restrict__ lp = lptr + uniform(pp->lptr_off);
  const int32_t nloc = static_cast<int32_t>(e0 - s0 + 1);

  double carry_v = 0.0;  // sum so far of the row continuing from earlier chunks
  bool carry_on = false;
  int32_t j0 = 0;         // first local row of the current chunk
  const int32_t lead = static_cast<int32_t>(s0 % K);  // align item groups to K
  // software pipeline: with PF == 1 the chunk's column indices and values are
  // loaded one chunk ahead; with PF == 2 they are loaded two chunks ahead and
  // the x gather runs one chunk ahead, so every wavefront keeps its gathers in
  // flight while it scans.
  const rsrc_t rx = make_rsrc(x, static_cast<uint32_t>(n) * static_cast<uint32_t>(sizeof(T)));
  const rsrc_t rl = make_rsrc(lp, static_cast<uint32_t>(R + 1 > 0 ? R + 1 : 0) * 4u);
  auto gather = [&](const int32_t(&c)[K], T(&xv)[K]) {
    // (index -1 and columns >= n read as 0 through the x resource)
#pragma unroll
    for (int t = 0; t < K; ++t)
      xv[t] = buf_load<T>(rx, static_cast<uint32_t>(c[t]) * static_cast<uint32_t>(sizeof(T)));
  };
  int32_t c_cur[K], c_nxt[K];
  V v_cur[K], v_nxt[K];
  T xv_cur[K], xv_nxt[K];
  load_items<V, K>(col, val, s0, -lead, nloc, c_cur, v_cur);
  if constexpr (PF == 2) {
    gather(c_cur, xv_cur);
    load_items<V, K>(col, val, s0, -lead + CH, nloc, c_nxt, v_nxt);
  }
  // PF == 2: a window of the local row pointer kept in registers: lw0 =
  // lp[j0 + lane] and lw1 = lp[j0 + 64 + lane]; each chunk loads the 64
  // words after it, and the window slides by the rows the chunk finished, so
  // a chunk needs no dependent pointer load unless 64 or more rows start
  // inside it.  (The register-lean PF == 1 loads lp[j0 + lane] per chunk.)
  int32_t lw0 = buf_load<int32_t>(rl, static_cast<uint32_t>(lane) * 4u);
  int32_t lw1 = PF == 2 ? buf_load<int32_t>(rl, static_cast<uint32_t>(kWave + lane) * 4u) : 0;
  for (int32_t cb = -lead; cb < nloc; cb += CH) {
    const int32_t cs = cb > 0 ? cb : 0;                 // first valid local position
    const int32_t ce = cb + CH < nloc ? cb + CH : nloc;  // one past the last
    // ---- 1. issue: the pointer words after the window, then the loads of
    //         later chunks, while this chunk's products are formed
    if constexpr (PF != 2) lw0 = buf_load<int32_t>(rl, static_cast<uint32_t>(j0 + lane) * 4u);
    const int32_t lpv0 = lw0;
    const int32_t lw2 =
        PF == 2 ? buf_load<int32_t>(rl, static_cast<uint32_t>(j0 + 2 * kWave + lane) * 4u) : 0;
    int32_t c_nn[K];
    V v_nn[K];
    if constexpr (PF == 2) {
      gather(c_nxt, xv_nxt);
      load_items<V, K>(col, val, s0, cb + 2 * CH, nloc, c_nn, v_nn);
    } else {
      gather(c_cur, xv_cur);
      load_items<V, K>(col, val, s0, cb + CH, nloc, c_nxt, v_nxt);
    }
    Acc prod[K];
#pragma unroll
    for (int t = 0; t < K; ++t) prod[t] = Tr::val(v_cur[t]) * static_cast<Acc>(xv_cur[t]);
    // ---- 2. rows that start inside the chunk: the first batch covers rows
    //         j0 .. j0+63 (lpv0); more start inside the chunk only with many
    //         short or empty rows
    int32_t jb = j0, cnt, lp_next;
    {
      const int32_t j = j0 + lane;
      const bool in = j <= R - 1 && lpv0 < ce;
      cnt = __popcll(__ballot(in));
      lp_next = read_lane(lpv0, cnt & (kWave - 1));
    }
    if (cnt == kWave) {
      // more than 64 rows start in the chunk (short or empty rows): wide
      // rounds from the next batch on
      jb += kWave;
      for (;;) {
        cnt = lp_wide_round<WL>(rl, jb, R, ce, lp_next, [](int32_t, int32_t, bool) {});
        if (cnt < WL * 4 * kWave) break;
        jb += WL * 4 * kWave;
      }
    }
    const int32_t j1 = jb + cnt - 1;  // last row starting before ce
    const bool cont = lp_next > ce;   // row j1 continues into the next chunk
    const bool one_batch = jb == j0;  // rows j0..j1 are the lanes of lpv0
    // next lane's pointer = lp[j + 1] while all rows sit in the first batch
    const int32_t lpv1 = __builtin_amdgcn_ds_bpermute(((lane + 1) & (kWave - 1)) << 2, lpv0);
    // this lane's row and its positions inside the chunk (first batch)
    const int32_t jl = j0 + lane;
    const int32_t aa = lpv0 > cs ? lpv0 : cs;
    const int32_t bl = jl == j1 ? lp_next : lpv1;
    const int32_t bb = bl < ce ? bl : ce;
    // a row is written (or its partial sum carried) once its total is known
    auto finish_row = [&](int32_t j, double tot) {
      if (j == j0 && carry_on) tot += carry_v;
      if (j == j1 && cont) return;
      if (j == 0 && sflag)
        carry[2 * static_cast<int64_t>(p)] = tot;
      else if (j == R - 1 && eflag)
        carry[2 * static_cast<int64_t>(p) + 1] = tot;
      else if (static_cast<uint32_t>(r0 + j) < static_cast<uint32_t>(m))
        store_y<T>(y, r0 + j, tot, alpha, beta, BETA0);
    };
    // ---- 3a. short rows (every row covers at most kShortRow positions of
    //          the chunk): each lane sums its own row's products from LDS
    const bool short_rows =
        one_batch && __ballot(jl <= j1 && bb - aa > kShortRow) == 0ull;
    double next_carry = 0.0;
    if (short_rows) {
#pragma unroll
      for (int t = 0; t < K; ++t) s_sum[lane * K + t] = prod[t];
      wave_lds_sync();
      // eight independent LDS reads per round (indices clamped into the
      // chunk; positions past the row add 0), summed in position order
      Acc acc = Acc(0);
      for (int32_t q = aa; q < bb; q += 8) {
        Acc v8[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int32_t qi = q + i < ce ? q + i : ce - 1;
          v8[i] = s_sum[qi - cb];
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) acc += q + i < bb ? v8[i] : Acc(0);
      }
      double tot = static_cast<double>(acc);
      if (jl <= j1) finish_row(jl, tot);
      if (cont) {  // the open row's sum so far, from the lane that holds it
        if (jl == j0 && carry_on) tot += carry_v;
        const int src = j1 - j0;
        const int64_t u = __builtin_bit_cast(int64_t, tot);
        const int lo = __builtin_amdgcn_readlane(static_cast<int>(u), src);
        const int hi = __builtin_amdgcn_readlane(static_cast<int>(u >> 32), src);
        next_carry = __builtin_bit_cast(double, (static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo));
      }
    } else {
      // ---- 3b. segmented scan: rows starting inside the chunk mark their
      //          first position; the scan restarts at every mark
#pragma unroll
      for (int w = 0; w < K / 4; ++w) reinterpret_cast<uint32_t *>(s_head)[lane * (K / 4) + w] = 0u;
      wave_lds_sync();
      for (int32_t jr = j0; jr <= j1; jr += RB * kWave) {
        int32_t v[RB];
#pragma unroll
        for (int u = 0; u < RB; ++u)
          v[u] = buf_load<int32_t>(rl, static_cast<uint32_t>(jr + u * kWave + lane) * 4u);
#pragma unroll
        for (int u = 0; u < RB; ++u) {
          const int32_t j = jr + u * kWave + lane;
          const int32_t pos = v[u] - cb;
          if (j > j0 && j <= j1 && pos > 0 && pos < CH) s_head[pos] = 1;
        }
      }
      wave_lds_sync();
      uint32_t hb[K / 4];
#pragma unroll
      for (int w = 0; w < K / 4; ++w) hb[w] = reinterpret_cast<const uint32_t *>(s_head)[lane * (K / 4) + w];
      Acc run[K];
      Acc r = Acc(0);
      bool any = false;
#pragma unroll
      for (int t = 0; t < K; ++t) {
        const bool h = (hb[t / 4] >> (8 * (t % 4))) & 0xffu;
        if (h) {
          r = Acc(0);
          any = true;
        }
        r += prod[t];
        run[t] = r;
      }
      Acc agg = r;
      int flg = any ? 1 : 0;
      wave_seg_scan<Acc>(agg, flg);
      const Acc cin = dpp<kDppWaveShr1>(agg);  // exclusive: lane 0 gets 0
      bool seen = false;
#pragma unroll
      for (int t = 0; t < K; ++t) {
        seen = seen || ((hb[t / 4] >> (8 * (t % 4))) & 0xffu);
        s_sum[lane * K + t] = seen ? run[t] : run[t] + cin;
      }
      wave_lds_sync();
      // a row's in-chunk sum is the scan value at its last position
      auto scanned = [&](int32_t a, int32_t b) {
        const int32_t a2 = a > cs ? a : cs, b2 = b < ce ? b : ce;
        return b2 > a2 ? static_cast<double>(s_sum[b2 - 1 - cb]) : 0.0;
      };
      if (one_batch) {
        if (jl <= j1) finish_row(jl, scanned(lpv0, bl));
      } else {
        for (int32_t jr = j0; jr <= j1; jr += RB * kWave) {
          int32_t a[RB], b[RB];
#pragma unroll
          for (int u = 0; u < RB; ++u) {
            const uint32_t j = static_cast<uint32_t>(jr + u * kWave + lane);
            a[u] = buf_load<int32_t>(rl, j * 4u);
            b[u] = buf_load<int32_t>(rl, (j + 1u) * 4u);
          }
#pragma unroll
          for (int u = 0; u < RB; ++u) {
            const int32_t j = jr + u * kWave + lane;
            if (j >= 0 && j <= j1) finish_row(j, scanned(a[u], b[u]));
          }
        }
      }
      if (cont) {
        const double last_tot = static_cast<double>(s_sum[ce - 1 - cb]);
        next_carry = last_tot + ((j1 == j0 && carry_on) ? carry_v : 0.0);
      }
    }
    carry_v = next_carry;
    carry_on = cont;
    {
      const int32_t j0n = cont ? j1 : j1 + 1;
      const int32_t d = j0n - j0;  // wave-uniform
      if constexpr (PF != 2) {
        // (reloaded at the next chunk's start)
      } else if (one_batch && d <= kWave) {
        // slide the window: lane L takes word j0n + L from lw0 / lw1 / lw2
        const int32_t src = lane + d;  // 0 .. 127
        const int addr = (src & (kWave - 1)) << 2;
        const int32_t a = __builtin_amdgcn_ds_bpermute(addr, lw0);
        const int32_t b = __builtin_amdgcn_ds_bpermute(addr, lw1);
        const int32_t c = __builtin_amdgcn_ds_bpermute(addr, lw2);
        lw0 = src < kWave ? a : b;
        lw1 = src < kWave ? b : c;
      } else {
        lw0 = buf_load<int32_t>(rl, static_cast<uint32_t>(j0n + lane) * 4u);
        lw1 = buf_load<int32_t>(rl, static_cast<uint32_t>(j0n + kWave + lane) * 4u);
      }
      j0 = j0n;
    }
#pragma unroll
    for (int t = 0; t < K; ++t) {
      c_cur[t] = c_nxt[t];
      v_cur[t] = v_nxt[t];
      if constexpr (PF == 2) {
        xv_cur[t] = xv_nxt[t];
        c_nxt[t] = c_nn[t];
        v_nxt[t] = v_nn[t];
      }
    }
    wave_lds_sync();  // s_sum / s_head are rewritten by the next chunk
  }
  // ---- empty rows after this partition up to the next one's first row
  const int32_t gap_lo = r0 + R;  // R == 0 for an empty partition
  const int32_t gap_hi_raw = p + 1 < np ? uniform(parts[p + 1].start_row) : m;
  const int32_t gap_hi = gap_hi_raw < m ? gap_hi_raw : m;
  if (!eflag) scale_rows<T>(y, gap_lo > 0 ? gap_lo : 0, gap_hi, beta, BETA0);
  if (p == 0) scale_rows<T>(y, 0, r0 < m ? r0 : m, beta, BETA0);
}

template <int VT, int K, bool BETA0, int PF>
__global__ __launch_bounds__(512) void spmv_csr_seg(
    const int32_t *__restrict__ col, const typename vt_traits<VT>::V *__restrict__ val,
    const msrep_part *__restrict__ parts, const int32_t *__restrict__ lptr, int32_t np,
    const typename vt_traits<VT>::T *__restrict__ x, typename vt_traits<VT>::T *__restrict__ y,
    int32_t m, int32_t n, double alpha, double beta, double *__restrict__ carry) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int wid = threadIdx.x / kWave;
  // one partition per wavefront, or (a grid of resident size) every W-th;
  // there is no block barrier, so wavefronts run independently
  const PartStride ps(np);
  for (int32_t p = ps.p; p < np; p += ps.step)
    csr_partition<VT, K, BETA0, PF>(col, val, parts, lptr, np, p, x, y, m, n, alpha, beta, carry,
                                    lds_raw + wid * seg_lds_per_wave<VT, K>());
}

// ---- boundary merge for the row-split formats (CSR, COO) ----
// The partial sums of split rows are combined as a segmented sum over the
// partitions in partition order (msRep Algorithm 3 merging step, Sec. 4.3).
// Partition q contributes two elements, in order: its head partial carry[2q]
// (the rest of the row split at its left edge, when start_flag is set) and
// its tail partial carry[2q+1] (the first piece of the row split at its right
// edge, when q holds that row's first piece).  The tail element starts a
// segment; a partition without start_flag, or one that ends on a row end,
// breaks the chain (a segment start with value 0).  The total of split row r
// is the segmented sum at the head element of the partition where r ends, and
// that partition's thread applies alpha and beta once.  Sums are kept as
// compensated pairs (s, c) combined with TwoSum.
struct MSeg {
  double s, c;  // value s + c
  int f;        // a segment starts in the range
};

// a before b
__device__ __forceinline__ MSeg mseg_cat(const MSeg &a, const MSeg &b) {
  if (b.f) return b;
  MSeg r;
  double e;
  two_sum(a.s, b.s, r.s, e);
  r.c = a.c + b.c + e;
  r.f = a.f;
  return r;
}

struct MPart {
  int32_t sr, er, sf, ef;  // start_row, end_row, start_flag, end_flag
};

__device__ __forceinline__ MPart mpart_load(const msrep_part *__restrict__ parts, int32_t q) {
  const int32_t *w = &parts[q].start_row;  // 8-byte aligned (40-byte records)
  return MPart{w[0], w[1], w[2], w[3]};
}

// The head and tail elements of one partition, combined.  An empty partition
// (end_row < start_row) is the identity.
__device__ __forceinline__ MSeg mpart_seg(const MPart &P, double head, double tail) {
  MSeg a{0.0, 0.0, 0};
  if (P.er < P.sr) return a;
  if (P.sf)
    a.s = head;
  else
    a.f = 1;
  const bool middle = P.sf && P.sr == P.er;  // inside one split row: its sum is the head
  if (!P.ef) return MSeg{0.0, 0.0, 1};
  if (!middle) return MSeg{tail, 0.0, 1};
  return a;
}

template <int CTRL, int ROWS>
__device__ __forceinline__ void mseg_step(MSeg &v) {
  MSeg p;
  p.s = dpp<CTRL, ROWS>(v.s);
  p.c = dpp<CTRL, ROWS>(v.c);
  p.f = dpp_i<CTRL, ROWS>(v.f);
  v = mseg_cat(p, v);  // lanes with no source get (0, 0, 0): the identity
}

constexpr int kMergeBlock = 256;  // partitions per block, one per thread
constexpr int kMergeLook = 4;     // partitions per thread in a look-back window
constexpr int kMergeWaves = kMergeBlock / kWave;

// Inclusive segmented scan across the 64 lanes.
__device__ __forceinline__ void wave_mseg_scan(MSeg &v) {
  mseg_step<kDppRowShr1, 0xF>(v);
  mseg_step<kDppRowShr2, 0xF>(v);
  mseg_step<kDppRowShr4, 0xF>(v);
  mseg_step<kDppRowShr8, 0xF>(v);
  mseg_step<kDppRowBcast15, 0xA>(v);
  mseg_step<kDppRowBcast31, 0xC>(v);
}

// Block-wide segmented scan in thread order: returns the block's total and
// sets excl to the sum of the threads before this one.  Ends with a barrier,
// so the LDS slots can be reused at once.
__device__ __forceinline__ MSeg block_mseg_scan(MSeg v, MSeg &excl, double *sh_s, double *sh_c,
                                                int *sh_f) {
  const int lane = lane_id(), wid = threadIdx.x / kWave;
  wave_mseg_scan(v);
  MSeg wex;  // exclusive within the wave
  wex.s = dpp<kDppWaveShr1>(v.s);
  wex.c = dpp<kDppWaveShr1>(v.c);
  wex.f = dpp_i<kDppWaveShr1>(v.f);
  if (lane == kWave - 1) {
    sh_s[wid] = v.s;
    sh_c[wid] = v.c;
    sh_f[wid] = v.f;
  }
  __syncthreads();
  MSeg pre{0.0, 0.0, 0}, tot{0.0, 0.0, 0};
#pragma unroll
  for (int w = 0; w < kMergeWaves; ++w) {
    const MSeg ww{sh_s[w], sh_c[w], sh_f[w]};
    if (w == wid) pre = tot;
    tot = mseg_cat(tot, ww);
  }
  excl = mseg_cat(pre, wex);
  __syncthreads();
  return tot;
}

template <typename T, bool BETA0>
__global__ __launch_bounds__(kMergeBlock) void merge_rows(const msrep_part *__restrict__ parts,
                                                          int32_t np,
                                                          const double *__restrict__ carry,
                                                          T *__restrict__ y, int32_t m,
                                                          double alpha, double beta,
                                                          int64_t ldy, int64_t cstride) {
  // several right-hand sides: column blockIdx.y of y (stride ldy between
  // rows) from its own block of carries
  carry += blockIdx.y * cstride;
  y += blockIdx.y;
  __shared__ double sh_s[kMergeWaves], sh_c[kMergeWaves];
  __shared__ int sh_f[kMergeWaves];
  const int t = threadIdx.x;
  const int32_t base = blockIdx.x * kMergeBlock;
  const int32_t q = base + t;
  MPart P{0, -1, 0, 0};
  double hd = 0.0, tl = 0.0;
  if (q < np) {
    P = mpart_load(parts, q);
    hd = carry[2 * static_cast<int64_t>(q)];
    tl = carry[2 * static_cast<int64_t>(q) + 1];
  }
  // the 64 partitions just before the block, loaded up front by wave 0: a
  // split row reaching into the block usually starts among them
  const int32_t near = base > kWave ? base - kWave : 0;
  MSeg look{0.0, 0.0, 0};
  if (t < kWave && near + t < base) {
    const int32_t qq = near + t;
    look = mpart_seg(mpart_load(parts, qq), carry[2 * static_cast<int64_t>(qq)],
                     carry[2 * static_cast<int64_t>(qq) + 1]);
  }

  MSeg excl;
  (void)block_mseg_scan(mpart_seg(P, hd, tl), excl, sh_s, sh_c, sh_f);
  const bool last = P.er >= P.sr && P.sf && !(P.ef && P.sr == P.er);  // a split row ends here
  MSeg at = mseg_cat(excl, MSeg{hd, 0.0, 0});  // segmented sum at the head element
  const bool need = last && !at.f;             // the row began before this block
  if (__syncthreads_or(need)) {
    // the segment open at the block's left edge: first the near window,
    // then windows of kMergeBlock * kMergeLook partitions further left
    // (block-uniform: every thread sees the same window totals)
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
    constexpr int32_t kSpan = kMergeBlock * kMergeLook;
    int32_t hi = near;
    while (hi > 0 && !acc.f) {
      const int32_t lo = hi > kSpan ? hi - kSpan : 0;
      MSeg w{0.0, 0.0, 0};
#pragma unroll
      for (int j = 0; j < kMergeLook; ++j) {
        const int32_t qq = lo + t * kMergeLook + j;
        if (qq < hi)
          w = mseg_cat(w, mpart_seg(mpart_load(parts, qq), carry[2 * static_cast<int64_t>(qq)],
                                    carry[2 * static_cast<int64_t>(qq) + 1]));
      }
      MSeg wex;
      acc = mseg_cat(block_mseg_scan(w, wex, sh_s, sh_c, sh_f), acc);
      hi = lo;
    }
    if (need) at = mseg_cat(acc, at);
  }
  if (!last) return;
  const int32_t r = P.sr;
  if (r < 0 || r >= m) return;
  const double tot = at.s + at.c;
  T *yr = y + static_cast<int64_t>(r) * ldy;
  *yr = static_cast<T>(BETA0 ? alpha * tot : alpha * tot + beta * static_cast<double>(*yr));
}

}  // namespace msrep
