// Multi-right-hand-side CSR SpMV (Y = alpha*A*X + beta*Y for k columns of X
// at once) over the same equal-nnz partitions as the single-vector pCSR path
// (msRep Algorithm 3): the product of Sec. 2.2 (Algorithm 1) applied to every
// column of a row-major block of vectors, the sparse-times-several-dense-
// vectors case that Sec. 2.3 groups with SpMV.
//
// X is n x k and Y is m x k, both row-major with leading dimensions ldx and
// ldy (elements), so the k values a nonzero multiplies are contiguous.  A pass
// covers NR columns (8, 4, 2 or 1), CPL of them per lane (1, or 2 for eight
// columns when X and Y keep column pairs aligned), so LPS = NR / CPL lanes
// share a slot.  One wavefront owns one partition and walks its nonzeros in
// chunks of 64.  Lane (q, cl) of a chunk takes slot q = lane / LPS, i.e. the
// LPS consecutive nonzeros q*LPS .. q*LPS+LPS-1, and columns cl*CPL ..
// cl*CPL+CPL-1: the LPS lanes of a slot read one X row as one contiguous
// NR-element segment, so a gather instruction touches 64/LPS rows of X
// instead of 64.  Per chunk:
//   1. rows of the chunk from the partition's local pointer (one row per lane
//      per round): a row starting inside the chunk writes its number at its
//      first position in LDS, a max-scan over the 64 positions gives every
//      position its row; empty rows get beta*Y here;
//   2. products val*X[col, c] in registers, summed sequentially over the
//      lane's LPS positions with restarts at row changes, then a segmented
//      scan across the slots (shifts of LPS, 2LPS, ... lanes);
//   3. the lane holding a row's last position in the chunk writes that row's
//      columns; the row open at the end of the chunk is carried (in FP64).
// Head and tail rows of a partition (start_flag / end_flag) go to the carry
// buffer, one block of 2*np doubles per column, which the boundary merge
// completes column by column.
#pragma once

#include <climits>
#include <type_traits>

#include "spmv_csr.hpp"

namespace msrep {

constexpr int kSpmmWaves = 4;  // wavefronts per block
constexpr int kSpmmMaxCols = 8;

// Lanes shifted up by d (lanes below d receive 0).
__device__ __forceinline__ int shift_up_i(int v, int d) {
  const int l = lane_id();
  const int r = __builtin_amdgcn_ds_bpermute((l >= d ? l - d : l) << 2, v);
  return l >= d ? r : 0;
}
template <typename A>
__device__ __forceinline__ A shift_up(A v, int d) {
  if constexpr (sizeof(A) == 8) {
    const int64_t u = __builtin_bit_cast(int64_t, v);
    const int lo = shift_up_i(static_cast<int>(u), d);
    const int hi = shift_up_i(static_cast<int>(u >> 32), d);
    return __builtin_bit_cast(A, (static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo));
  } else {
    return __builtin_bit_cast(A, shift_up_i(__builtin_bit_cast(int, v), d));
  }
}

// Value of lane src (per lane) of v.
template <typename A>
__device__ __forceinline__ A lane_pick(A v, int src) {
  if constexpr (sizeof(A) == 8) {
    const int64_t u = __builtin_bit_cast(int64_t, v);
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, static_cast<int>(u));
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, static_cast<int>(u >> 32));
    return __builtin_bit_cast(A, (static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo));
  } else if constexpr (sizeof(A) == 4) {
    return __builtin_bit_cast(A, __builtin_amdgcn_ds_bpermute(src << 2, __builtin_bit_cast(int, v)));
  } else {
    static_assert(sizeof(A) == 2, "2, 4 or 8 bytes");
    const int w = static_cast<int>(__builtin_bit_cast(uint16_t, v));
    return __builtin_bit_cast(A, static_cast<uint16_t>(__builtin_amdgcn_ds_bpermute(src << 2, w)));
  }
}

// One element stored at byte offset `off` (dropped by the hardware when
// outside the resource).
template <typename E>
__device__ __forceinline__ void buf_store(rsrc_t r, uint32_t off, E v) {
  if constexpr (sizeof(E) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 0);
}
// CPL consecutive elements at byte offset `off` (one 8- or 16-byte access;
// `off` a multiple of its size).
template <typename T, int CPL>
__device__ __forceinline__ void buf_load_n(rsrc_t r, uint32_t off, T (&out)[CPL]) {
  if constexpr (CPL == 1) {
    out[0] = buf_load<T>(r, off);
  } else {
    static_assert(CPL == 2, "one or two elements");
    // (elements are copied out of the vector into scalars before the bit
    // casts: hipcc has folded a bit cast of `w.y` into one of `w.x`)
    if constexpr (sizeof(T) == 8) {
      const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
      const uint64_t a = static_cast<uint64_t>(static_cast<uint32_t>(w[0])) |
                         (static_cast<uint64_t>(static_cast<uint32_t>(w[1])) << 32);
      const uint64_t b = static_cast<uint64_t>(static_cast<uint32_t>(w[2])) |
                         (static_cast<uint64_t>(static_cast<uint32_t>(w[3])) << 32);
      out[0] = __builtin_bit_cast(T, a);
      out[1] = __builtin_bit_cast(T, b);
    } else {
      const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
      const uint32_t a = w[0], b = w[1];
      out[0] = __builtin_bit_cast(T, a);
      out[1] = __builtin_bit_cast(T, b);
    }
  }
}
template <typename T, int CPL>
__device__ __forceinline__ void buf_store_n(rsrc_t r, uint32_t off, const T (&v)[CPL]) {
  if constexpr (CPL == 1) {
    buf_store<T>(r, off, v[0]);
  } else if constexpr (sizeof(T) == 8) {
    const uint64_t a = __builtin_bit_cast(uint64_t, v[0]), b = __builtin_bit_cast(uint64_t, v[1]);
    const u32x4 w = {static_cast<uint32_t>(a), static_cast<uint32_t>(a >> 32),
                     static_cast<uint32_t>(b), static_cast<uint32_t>(b >> 32)};
    __builtin_amdgcn_raw_buffer_store_b128(w, r, off, 0, 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b64(
        u32x2{__builtin_bit_cast(uint32_t, v[0]), __builtin_bit_cast(uint32_t, v[1])}, r, off, 0, 0);
  }
}
constexpr uint32_t kNoStore = 0xFFFFFFF0u;  // offsets down to kNoStore - 511 are past every resource

// Rows [lo, hi) x columns [0, NR) get beta*Y (0 when beta == 0), lanes
// striding over the elements.
template <typename T, int NR>
__device__ __forceinline__ void spmm_scale_rows(T *__restrict__ Y, int64_t ldy, int32_t lo,
                                                int32_t hi, double beta, bool beta0) {
  if (hi <= lo) return;
  const int64_t cnt = static_cast<int64_t>(hi - lo) * NR;
  for (int64_t e = lane_id(); e < cnt; e += kWave) {
    const int64_t at = static_cast<int64_t>(lo + static_cast<int32_t>(e / NR)) * ldy + e % NR;
    Y[at] = beta0 ? static_cast<T>(0) : static_cast<T>(beta * static_cast<double>(Y[at]));
  }
}

// Partition p of one pass: NR columns of X (n rows of ldx) into Y (m rows of
// ldy), head and tail carries of column c at carry + c*cstride + 2p.
// s_mark and s_rows: 64 ints of LDS each, the wavefront's own.
template <int VT, int NR, bool BETA0, int CPL>
__device__ __forceinline__ void spmm_partition(
    const int32_t *__restrict__ col, const typename vt_traits<VT>::V *__restrict__ val,
    const msrep_part *__restrict__ parts, const int32_t *__restrict__ lptr, int32_t np, int32_t p,
    const typename vt_traits<VT>::T *__restrict__ X, int64_t ldx,
    typename vt_traits<VT>::T *__restrict__ Y, int64_t ldy, int32_t m, double alpha,
    double beta, double *__restrict__ carry, int64_t cstride, uint32_t xbytes, uint32_t ybytes,
    int32_t *s_mark, int32_t *s_rows) {
  using Tr = vt_traits<VT>;
  using V = typename Tr::V;
  using T = typename Tr::T;
  using Acc = typename Tr::A;
  static_assert(NR == 1 || NR == 2 || NR == 4 || NR == 8, "columns per pass");
  static_assert(CPL == 1 || (CPL == 2 && NR >= 2), "one or two columns per lane");
  constexpr int LPS = NR / CPL;   // lanes per slot
  constexpr int U = LPS;          // positions per slot
  constexpr int G = kWave / LPS;  // slots per chunk
  const int lane = lane_id();
  const int q = lane / LPS, cl = lane % LPS;  // slot, and the lane's first column / CPL
  // byte offsets of X and Y elements (32-bit)
  const uint32_t xrow = static_cast<uint32_t>(ldx) * sizeof(T), xcol = cl * CPL * sizeof(T);
  const uint32_t yrow = static_cast<uint32_t>(ldy) * sizeof(T);
  {
    const msrep_part *pp = parts + p;
    const int64_t s0 = uniform(pp->start_idx);
    const int64_t e0 = uniform(pp->end_idx);
    const int32_t r0 = uniform(pp->start_row);
    const int32_t R = uniform(pp->end_row) - r0 + 1;
    const int32_t sflag = uniform(pp->start_flag);
    const int32_t eflag = uniform(pp->end_flag);
    const int32_t *__restrict__ lp = lptr + uniform(pp->lptr_off);
    const int32_t nloc = R > 0 ? static_cast<int32_t>(e0 - s0 + 1) : 0;
    const rsrc_t rl = make_rsrc(lp, static_cast<uint32_t>(R + 1 > 0 ? R + 1 : 0) * 4u);
    const rsrc_t ry = make_rsrc(Y, ybytes);  // X and Y are below 4 GiB (checked by the host)
    const rsrc_t rx = make_rsrc(X, xbytes);
    // the lane's columns' head and tail carries
    double *cp = carry + static_cast<int64_t>(cl * CPL) * cstride + 2 * static_cast<int64_t>(p);
    double cv[CPL];  // the lane's columns of the row continuing from the previous chunk
#pragma unroll
    for (int e = 0; e < CPL; ++e) cv[e] = 0.0;
    bool con = false;
    int32_t j0 = 0;   // first local row of the chunk
    // software pipeline: every lane loads one nonzero (column index and
    // value) of the chunk after next, coalesced, and the X gather of the next
    // chunk is issued before this chunk's rows are worked out.  Lane (q, cl)
    // takes the index and value of position q*U + u from lane q*U + u.
    auto load_item = [&](int32_t cbx, int32_t &ci, V &vi) {
      const int32_t left = nloc - cbx;
      const uint32_t cnt = static_cast<uint32_t>(left <= 0 ? 0 : left < kWave ? left : kWave);
      const int64_t off = left <= 0 ? 0 : s0 + cbx;  // (nothing is read when cnt == 0)
      const rsrc_t rc = make_rsrc(col + off, cnt * 4u);
      const rsrc_t rv = make_rsrc(val + off, cnt * static_cast<uint32_t>(sizeof(V)));
      ci = buf_load<int32_t, kNt>(rc, static_cast<uint32_t>(lane) * 4u);
      vi = buf_load<V, kNt>(rv, static_cast<uint32_t>(lane) * static_cast<uint32_t>(sizeof(V)));
      // the byte offset of the item's X row; past the partition an offset
      // past X's resource, so x = 0 and value = 0 there and the product is
      // exactly 0
      ci = static_cast<uint32_t>(lane) < cnt ? static_cast<int32_t>(static_cast<uint32_t>(ci) * xrow)
                                              : static_cast<int32_t>(kNoStore - 256u);
    };
    auto gather = [&](int32_t ci, T(&xv)[U][CPL]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t ro = static_cast<uint32_t>(lane_pick(ci, q * U + u));  // X row offset
        buf_load_n<T, CPL>(rx, ro + xcol, xv[u]);
      }
    };
    // two sets of pipeline registers used in turn by consecutive chunks (no
    // copies between them, which would wait for the loads in flight)
    int32_t cA = 0, cB = 0;
    V vA = V(0), vB = V(0);
    T xvA[U][CPL], xvB[U][CPL];
    int32_t a0 = 0, b0 = 0;  // first round of row pointers of the chunk
    if (nloc > 0) {
      a0 = buf_load<int32_t>(rl, static_cast<uint32_t>(lane) * 4u);
      b0 = buf_load<int32_t>(rl, static_cast<uint32_t>(lane + 1) * 4u);
      int32_t c0;
      load_item(0, c0, vA);
      gather(c0, xvA);
      V vdummy;
      load_item(kWave, cA, vdummy);  // (the value is loaded again one chunk later)
      // as many (dropped) stores as a chunk issues, so that the memory
      // operations after each load are as many here as in the loop
      T zero[CPL];
#pragma unroll
      for (int e = 0; e < CPL; ++e) zero[e] = T(0);
#pragma unroll
      for (int u = 0; u < U; ++u) buf_store_n<T, CPL>(ry, kNoStore - 32u * (u + 1), zero);
    }
    // one chunk at cb: X values xv_use and values v_use of this chunk in
    // hand, c_use the column indices of the next one; fills xv_fill (next
    // chunk's X), v_fill (next chunk's values) and c_fill (the chunk after)
    auto chunk = [&](int32_t cb, T(&xv_use)[U][CPL], T(&xv_fill)[U][CPL], V &v_use, V &v_fill,
                     int32_t &c_use, int32_t &c_fill) {
      const int32_t ce = cb + kWave < nloc ? cb + kWave : nloc;
      const int32_t nv = ce - cb;  // valid positions of the chunk
      // ---- 1. rows: marks at the first position of every row starting in the chunk
      s_mark[lane] = 0;
      wave_lds_sync();
      auto visit = [&](int32_t j, int32_t a, int32_t b) {
        const bool in = j <= R - 1 && a < ce;
        if (in && a < b && j > j0 && a >= cb) s_mark[a - cb] = j;
        if (in && a == b) {  // empty row (never a head or tail row)
          const int64_t base = static_cast<int64_t>(r0 + j) * ldy;
#pragma unroll
          for (int t = 0; t < NR; ++t)
            Y[base + t] = BETA0 ? static_cast<T>(0)
                                : static_cast<T>(beta * static_cast<double>(Y[base + t]));
        }
        return in;
      };
      int32_t jb = j0;
      int cnt = __popcll(__ballot(visit(j0 + lane, a0, b0)));
      int32_t lp_next = read_lane(a0, cnt & (kWave - 1));
      while (cnt == kWave) {  // 64 rows start in the chunk: further rounds
        jb += kWave;
        const int32_t j = jb + lane;
        const int32_t a = buf_load<int32_t>(rl, static_cast<uint32_t>(j) * 4u);
        const int32_t b = buf_load<int32_t>(rl, static_cast<uint32_t>(j + 1) * 4u);
        cnt = __popcll(__ballot(visit(j, a, b)));
        lp_next = read_lane(a, cnt & (kWave - 1));
      }
      // lp_next = lp[j1 + 1], which exists (j1 + 1 <= R)
      const int32_t j1 = jb + cnt - 1;
      const bool cont = lp_next > ce;  // row j1 continues into the next chunk
      const int32_t j0n = cont ? j1 : j1 + 1;
      // ---- the next chunk's row pointers and X gather, the items of the
      //      chunk after it (past the partition: nothing is read)
      a0 = buf_load<int32_t>(rl, static_cast<uint32_t>(j0n + lane) * 4u);
      b0 = buf_load<int32_t>(rl, static_cast<uint32_t>(j0n + lane + 1) * 4u);
      gather(c_use, xv_fill);
      {
        V vn;
        int32_t cn;
        load_item(cb + kWave, cn, vn);  // next chunk's values
        v_fill = vn;
        load_item(cb + 2 * kWave, c_fill, vn);  // the column indices of the chunk after
        (void)cn;
      }
      wave_lds_sync();
      const int32_t mk = s_mark[lane];
      int32_t rr = wave_max_scan_nonneg(mk);
      rr = rr > j0 ? rr : j0;
      // positions past the chunk's end get a row that no row equals
      constexpr int32_t kNoRow = INT32_MIN;
      s_rows[lane] = lane < nv ? rr : kNoRow;
      wave_lds_sync();
      int32_t rw[U + 1];
#pragma unroll
      for (int u = 0; u < U; ++u) rw[u] = s_rows[q * U + u];
      rw[U] = q + 1 < G ? s_rows[(q + 1) * U] : kNoRow;
      const int32_t rprev = q > 0 ? s_rows[q * U - 1] : rw[0];
      wave_lds_sync();  // s_mark / s_rows are rewritten by the next chunk
      // ---- 2. products, sequential segmented sums over the lane's positions
      Acc run[U][CPL];
      bool seen[U];
      Acc acc[CPL];
#pragma unroll
      for (int e = 0; e < CPL; ++e) acc[e] = Acc(0);
      bool any = false;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t P = q * U + u;
        const bool h = rw[u] != (u == 0 ? rprev : rw[u - 1]);
        if (h) {
#pragma unroll
          for (int e = 0; e < CPL; ++e) acc[e] = Acc(0);
          any = true;
        }
        const V vu = lane_pick(v_use, P);
#pragma unroll
        for (int e = 0; e < CPL; ++e) {
          acc[e] += Tr::val(vu) * static_cast<Acc>(xv_use[u][e]);
          run[u][e] = acc[e];
        }
        seen[u] = any;
      }
      // segmented scan of the slot totals across slots (stride LPS lanes).
      // FP64: the sum carried from the previous chunk enters as slot 0's
      // incoming value; FP32 keeps it apart in FP64 and adds it at the end.
      constexpr bool kFold = sizeof(Acc) == 8;
      Acc cvin[CPL], agg[CPL], cin[CPL];
#pragma unroll
      for (int e = 0; e < CPL; ++e) {
        cvin[e] = kFold && con ? static_cast<Acc>(cv[e]) : Acc(0);
        agg[e] = (q == 0 && !any) ? acc[e] + cvin[e] : acc[e];
      }
      int f = any ? 1 : 0;
#pragma unroll
      for (int d = LPS; d < kWave; d *= 2) {
        Acc pv[CPL];
#pragma unroll
        for (int e = 0; e < CPL; ++e) pv[e] = shift_up(agg[e], d);
        const int pf = shift_up_i(f, d);
#pragma unroll
        for (int e = 0; e < CPL; ++e)
          if (!f) agg[e] += pv[e];
        f |= pf;
      }
#pragma unroll
      for (int e = 0; e < CPL; ++e) {
        const Acc cin0 = shift_up(agg[e], LPS);  // the open segment up to the previous slot
        cin[e] = q == 0 ? cvin[e] : cin0;
      }
      // ---- 3. rows ending at this lane's positions: one buffer store per
      //         position on every lane (dropped where no row ends), so the
      //         number of stores after the next chunks' loads is fixed and
      //         waiting for those loads never waits for these stores
      // (the partial sums of the partition's first and last rows, when they
      // are split, are kept aside and stored after the loop: at most one
      // position of a lane holds each)
      double hval[CPL], tval[CPL];
#pragma unroll
      for (int e = 0; e < CPL; ++e) hval[e] = tval[e] = 0.0;
      bool hset = false, tset = false;
      const int32_t skip_row = cont ? j1 : kNoRow + 1;  // the open row is carried, not written
      // only the chunks holding the partition's first or last row can hold a
      // partial row; the others take the short path
      const bool edge = (sflag && j0 == 0) || (eflag && j1 == R - 1);
      auto finish = [&](auto edge_c) {
        constexpr bool EDGE = decltype(edge_c)::value;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int32_t rj = rw[u];
          const bool done = rw[u + 1] != rj && rj != skip_row;
          double tot[CPL];
#pragma unroll
          for (int e = 0; e < CPL; ++e) {
            tot[e] = static_cast<double>(seen[u] ? run[u][e] : run[u][e] + cin[e]);
            if (!kFold && rj == j0 && con) tot[e] += cv[e];
          }
          bool to_y = done;
          if constexpr (EDGE) {
            const bool head_c = done && rj == 0 && sflag;
            const bool tail_c = done && !head_c && rj == R - 1 && eflag;
#pragma unroll
            for (int e = 0; e < CPL; ++e) {
              hval[e] = head_c ? tot[e] : hval[e];
              tval[e] = tail_c ? tot[e] : tval[e];
            }
            hset = hset || head_c;
            tset = tset || tail_c;
            to_y = done && !head_c && !tail_c;
          }
          const uint32_t off = to_y ? static_cast<uint32_t>(r0 + rj) * yrow + xcol : kNoStore;
          T old[CPL], out[CPL];
          if (!BETA0) buf_load_n<T, CPL>(ry, off, old);
#pragma unroll
          for (int e = 0; e < CPL; ++e) {
            double o = alpha * tot[e];
            if (!BETA0) o += beta * static_cast<double>(old[e]);
            out[e] = static_cast<T>(o);
          }
          buf_store_n<T, CPL>(ry, off, out);
        }
      };
      if (edge) {
        finish(std::true_type{});
#pragma unroll
        for (int e = 0; e < CPL; ++e) {
          if (hset) cp[e * cstride] = hval[e];
          if (tset) cp[e * cstride + 1] = tval[e];
        }
      } else {
        finish(std::false_type{});
      }
      if (cont) {  // the lane's columns of the open row, from the lane holding the chunk's last position
        const int ul = (nv - 1) % U;
        const int src = ((nv - 1) / U) * LPS + cl;
#pragma unroll
        for (int e = 0; e < CPL; ++e) {
          Acc lv = Acc(0);
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (u == ul) lv = seen[u] ? run[u][e] : run[u][e] + cin[e];
          const double open = static_cast<double>(lane_pick(lv, src));
          cv[e] = open + ((!kFold && j1 == j0 && con) ? cv[e] : 0.0);
        }
      }
      con = cont;
      j0 = j0n;
    };
    for (int32_t cb = 0; cb < nloc; cb += 2 * kWave) {
      chunk(cb, xvA, xvB, vA, vB, cA, cB);
      if (cb + kWave >= nloc) break;
      chunk(cb + kWave, xvB, xvA, vB, vA, cB, cA);
    }
    // ---- empty rows after this partition up to the next one's first row
    const int32_t gap_lo = r0 + R;
    const int32_t gap_hi_raw = p + 1 < np ? uniform(parts[p + 1].start_row) : m;
    const int32_t gap_hi = gap_hi_raw < m ? gap_hi_raw : m;
    if (!eflag) spmm_scale_rows<T, NR>(Y, ldy, gap_lo > 0 ? gap_lo : 0, gap_hi, beta, BETA0);
    if (p == 0) spmm_scale_rows<T, NR>(Y, ldy, 0, r0 < m ? r0 : m, beta, BETA0);
  }
}

template <int VT, int NR, bool BETA0, int CPL>
__global__ __launch_bounds__(kSpmmWaves * kWave) __attribute__((amdgpu_waves_per_eu(4))) void spmm_csr(
    const int32_t *__restrict__ col, const typename vt_traits<VT>::V *__restrict__ val,
    const msrep_part *__restrict__ parts, const int32_t *__restrict__ lptr, int32_t np,
    const typename vt_traits<VT>::T *__restrict__ X, int64_t ldx,
    typename vt_traits<VT>::T *__restrict__ Y, int64_t ldy, int32_t m, double alpha,
    double beta, double *__restrict__ carry, int64_t cstride, uint32_t xbytes, uint32_t ybytes) {
  __shared__ int32_t s_mark_all[kSpmmWaves][kWave];
  __shared__ int32_t s_rows_all[kSpmmWaves][kWave];
  const int wid = threadIdx.x / kWave;
  const PartStride ps(np);
  for (int32_t p = ps.p; p < np; p += ps.step)
    spmm_partition<VT, NR, BETA0, CPL>(col, val, parts, lptr, np, p, X, ldx, Y, ldy, m, alpha,
                                       beta, carry, cstride, xbytes, ybytes, s_mark_all[wid],
                                       s_rows_all[wid]);
}

}  // namespace msrep
