// Wave-per-partition segmented SpMV on row-sorted COO (pCOO, msRep
// Algorithm 7).  Same chunking as the CSR kernel, but the row of every
// nonzero is stored, so segment boundaries come straight from comparing
// neighbouring row indices: no local pointer and no search.  The lane that
// holds a segment's last nonzero writes the row's y (or its partial sum to
// the carry buffer for a row split across partitions), and the lane holding
// a segment's first nonzero writes beta*y for the empty rows between it and
// the previous segment.  With beta == 0, a chunk spanning more than 2*64*K
// rows (mostly empty ones in power-law matrices) is cleared by the whole
// wavefront first, which beats one lane per gap.
#pragma once

#include "spmv_csr.hpp"

namespace msrep {

// Row indices of a lane's K items (see load_items); items before the
// partition take its first row and items past its end its last row, so they
// join the first / last segment with a zero product.
template <int K>
__device__ __forceinline__ void load_rows(const int32_t *__restrict__ row_idx, int64_t s0,
                                          int32_t cb, int32_t nloc, int32_t r0, int32_t rE,
                                          int32_t (&row)[K]) {
  constexpr int CH = kWave * K;
  const int32_t span = nloc - cb < CH ? nloc - cb : CH;
  const rsrc_t rr = make_rsrc(row_idx + s0 + cb, static_cast<uint32_t>(span > 0 ? span : 0) * 4u);
  const uint32_t l = static_cast<uint32_t>(lane_id() * K);
  buf_load_vec<int32_t, K, kNt>(rr, l * 4u, row);
#pragma unroll
  for (int t = 0; t < K; ++t) {
    const int32_t q = cb + static_cast<int32_t>(l) + t;
    row[t] = q < 0 ? r0 : (q >= nloc ? rE : row[t]);
  }
}

template <int VT, int K>
constexpr size_t coo_lds_per_wave() {
  return 16;  // one FP64 slot: the sum carried into the next chunk
}

// One wavefront processes partition p of a row-sorted COO matrix; s_carry is
// this wavefront's LDS slot.
template <int VT, int K, bool BETA0>
__device__ __forceinline__ void coo_partition(
    const int32_t *__restrict__ row_idx, const int32_t *__restrict__ col,
    const typename vt_traits<VT>::V *__restrict__ val, const msrep_part *__restrict__ parts,
    int32_t np, int32_t p, const typename vt_traits<VT>::T *__restrict__ x,
    typename vt_traits<VT>::T *__restrict__ y, int32_t m, int32_t n, double alpha, double beta,
    double *__restrict__ carry, double *s_carry) {
  using Tr = vt_traits<VT>;
  using V = typename Tr::V;
  using T = typename Tr::T;
  using Acc = typename Tr::A;
  constexpr int CH = kWave * K;
  const int lane = lane_id();

  const msrep_part *pp = parts + p;
  const int64_t s0 = uniform(pp->start_idx);
  const int64_t e0 = uniform(pp->end_idx);
  const int32_t r0 = uniform(pp->start_row);
  const int32_t rE = uniform(pp->end_row);
  const int32_t sflag = uniform(pp->start_flag);
  const int32_t eflag = uniform(pp->end_flag);
  const int32_t nloc = static_cast<int32_t>(e0 - s0 + 1);

  double carry_v = 0.0;  // partial sum of the row continuing from the last chunk
  bool carry_on = false;
  const int32_t lead = static_cast<int32_t>(s0 % K);
  const rsrc_t rx = make_rsrc(x, static_cast<uint32_t>(n) * static_cast<uint32_t>(sizeof(T)));
  auto gather = [&](const int32_t(&c)[K], T(&xv)[K]) {
    // (index -1 and columns >= n read as 0 through the x resource)
#pragma unroll
    for (int t = 0; t < K; ++t)
      xv[t] = buf_load<T>(rx, static_cast<uint32_t>(c[t]) * static_cast<uint32_t>(sizeof(T)));
  };
  // software pipeline: rows, columns and values two chunks ahead, the x
  // gather one chunk ahead.  The rows next to a chunk (the last one before
  // it, the first one after it) come from the neighbouring chunks' registers.
  int32_t row_cur[K], c_cur[K], row_nxt[K], c_nxt[K];
  V v_cur[K], v_nxt[K];
  T xv_cur[K];
  load_items<V, K>(col, val, s0, -lead, nloc, c_cur, v_cur);
  load_rows<K>(row_idx, s0, -lead, nloc, r0, rE, row_cur);
  gather(c_cur, xv_cur);
  load_items<V, K>(col, val, s0, -lead + CH, nloc, c_nxt, v_nxt);
  load_rows<K>(row_idx, s0, -lead + CH, nloc, r0, rE, row_nxt);
  int32_t before = -1;  // row of the position just before the chunk (none for the first)
  for (int32_t cb = -lead; cb < nloc; cb += CH) {
    const int32_t cs = cb > 0 ? cb : 0;
    const int32_t ce = cb + CH < nloc ? cb + CH : nloc;
    const int32_t q0 = cb + lane * K;
    T xv_nxt[K];
    gather(c_nxt, xv_nxt);
    int32_t row_nn[K], c_nn[K];
    V v_nn[K];
    load_items<V, K>(col, val, s0, cb + 2 * CH, nloc, c_nn, v_nn);
    load_rows<K>(row_idx, s0, cb + 2 * CH, nloc, r0, rE, row_nn);
    // row of the position just after the chunk: the next chunk's first item
    const int32_t after = ce < nloc ? __builtin_amdgcn_readlane(row_nxt[0], 0) : -1;
    // a chunk over a long run of rows (most of them empty): the wavefront
    // clears the rows between its first and last row, then its lanes store
    // only the rows that hold nonzeros
    const int32_t last_row_c = __builtin_amdgcn_readlane(row_cur[K - 1], kWave - 1);
    const int32_t fill_lo = cb > 0 ? before + 1 : r0;
    const bool fill = BETA0 && last_row_c - fill_lo > 2 * CH;
    if (fill) {
      const int32_t hi = last_row_c < m ? last_row_c : m;
      for (int32_t g = (fill_lo > 0 ? fill_lo : 0) + lane; g < hi; g += kWave) y[g] = T(0);
      __builtin_amdgcn_s_waitcnt(0x0F70);  // the clears land before the rows' values
    }
    int32_t row[K];
    Acc prod[K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
      row[t] = row_cur[t];
      prod[t] = Tr::val(v_cur[t]) * static_cast<Acc>(xv_cur[t]);
    }
    // previous / next row of every item
    const int32_t up = shfl_up_i(row[K - 1], 1);
    const int32_t prev0 = lane == 0 ? before : up;
    const int32_t dn = __builtin_amdgcn_ds_bpermute(((lane + 1) & (kWave - 1)) << 2, row[0]);
    // ---- segmented scan (heads where the row changes inside the chunk)
    bool head[K];
    Acc run[K];
    Acc r = Acc(0);
    bool any = false;
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const int32_t q = q0 + t;
      const int32_t pr = t == 0 ? prev0 : row[t - 1];
      head[t] = q > cs && q < ce && row[t] != pr;
      if (head[t]) {
        r = Acc(0);
        any = true;
      }
      r += prod[t];
      run[t] = r;
    }
    Acc agg = r;
    int flg = any ? 1 : 0;
    wave_seg_scan<Acc>(agg, flg);
    const Acc cin = dpp<kDppWaveShr1>(agg);   // exclusive: lane 0 gets 0
    const int fin = dpp_i<kDppWaveShr1>(flg);
    // items before the lane's first head continue the segment of earlier
    // lanes (cin); only the chunk's first segment continues the carried row
    bool seen = false;
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const int32_t q = q0 + t;
      seen = seen || head[t];
      const bool first_seg = !seen && fin == 0;
      const double tot = static_cast<double>(seen ? run[t] : run[t] + cin) +
                         ((first_seg && carry_on) ? carry_v : 0.0);
      if (q < cs || q >= ce) continue;
      const int32_t rr = row[t];
      const int32_t pr = t == 0 ? prev0 : row[t - 1];
      // empty rows between the previous nonzero's row and this one
      if (!fill && (q > 0) && rr > pr + 1) {
        const int32_t lo = pr + 1 > 0 ? pr + 1 : 0, hi = rr < m ? rr : m;
        for (int32_t g = lo; g < hi; ++g)
          y[g] = BETA0 ? T(0) : static_cast<T>(beta * static_cast<double>(y[g]));
      }
      const int32_t nx = t + 1 < K ? row[t + 1] : dn;
      const bool end = q == ce - 1 || rr != nx;
      if (!end) continue;
      if (q == ce - 1 && after == rr) {
        *s_carry = tot;  // open row: carried into the next chunk
      } else if (rr == r0 && sflag) {
        carry[2 * static_cast<int64_t>(p)] = tot;
      } else if (rr == rE && eflag) {
        carry[2 * static_cast<int64_t>(p) + 1] = tot;
      } else if (static_cast<uint32_t>(rr) < static_cast<uint32_t>(m)) {
        store_y<T>(y, rr, tot, alpha, beta, BETA0);
      }
    }
    wave_lds_sync();
    // the chunk's last position is lane 63's last item when the chunk is full
    const int32_t last_row = __builtin_amdgcn_readlane(row[K - 1], kWave - 1);
    carry_on = ce < nloc && after == last_row;
    carry_v = carry_on ? *s_carry : 0.0;
    before = last_row;
#pragma unroll
    for (int t = 0; t < K; ++t) {
      row_cur[t] = row_nxt[t];
      c_cur[t] = c_nxt[t];
      v_cur[t] = v_nxt[t];
      xv_cur[t] = xv_nxt[t];
      row_nxt[t] = row_nn[t];
      c_nxt[t] = c_nn[t];
      v_nxt[t] = v_nn[t];
    }
    wave_lds_sync();
  }
  const int32_t gap_lo = nloc > 0 ? rE + 1 : r0;
  const int32_t gap_hi_raw = p + 1 < np ? uniform(parts[p + 1].start_row) : m;
  const int32_t gap_hi = gap_hi_raw < m ? gap_hi_raw : m;
  if (!eflag) scale_rows<T>(y, gap_lo > 0 ? gap_lo : 0, gap_hi, beta, BETA0);
  if (p == 0) scale_rows<T>(y, 0, r0 < m ? r0 : m, beta, BETA0);
}

// Wavefronts striding over the partitions (see PartStride).
template <int VT, int K, bool BETA0>
__global__ __launch_bounds__(512) void spmv_coo_seg(
    const int32_t *__restrict__ row_idx, const int32_t *__restrict__ col,
    const typename vt_traits<VT>::V *__restrict__ val, int64_t nnz,
    const msrep_part *__restrict__ parts, int32_t np,
    const typename vt_traits<VT>::T *__restrict__ x, typename vt_traits<VT>::T *__restrict__ y,
    int32_t m, int32_t n, double alpha, double beta, double *__restrict__ carry) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  (void)nnz;
  const int wid = threadIdx.x / kWave;
  double *s_carry = reinterpret_cast<double *>(lds_raw + wid * coo_lds_per_wave<VT, K>());
  const PartStride ps(np);
  for (int32_t p = ps.p; p < np; p += ps.step)
    coo_partition<VT, K, BETA0>(row_idx, col, val, parts, np, p, x, y, m, n, alpha, beta, carry,
                                s_carry);
}

}  // namespace msrep
