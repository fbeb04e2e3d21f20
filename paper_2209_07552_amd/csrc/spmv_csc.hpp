// Wave-per-partition CSC scatter SpMV (pCSC, msRep Algorithm 5).  Every
// nonzero of column j adds val * x[j] to y[row]; the paper merges the
// partitions' full-length partial vectors by summing them (Sec. 4.3), which on
// one GPU is an atomic add into y after y <- beta*y.  The column of each
// nonzero comes from the partition's local column pointer: columns that start
// inside a chunk store their index at their first position in LDS and a
// max-scan carries it forward.  FP32/BF16 values accumulate into an FP64
// workspace that a final pass rounds into y once.
#pragma once

#include "spmv_csr.hpp"

namespace msrep {

template <int K>
constexpr size_t csc_lds_per_wave() {
  return align_up(kWave * K * sizeof(int32_t), 16);
}

template <typename T>
__global__ __launch_bounds__(256) void scale_y(T *__restrict__ y, int32_t m, double beta) {
  for (int64_t r = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; r < m;
       r += int64_t(gridDim.x) * blockDim.x)
    y[r] = beta == 0.0 ? T(0) : static_cast<T>(beta * static_cast<double>(y[r]));
}

__global__ __launch_bounds__(256) void zero_f64(double *__restrict__ a, int64_t n) {
  for (int64_t r = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; r < n;
       r += int64_t(gridDim.x) * blockDim.x)
    a[r] = 0.0;
}

// y = beta*y + alpha*acc, rounded once (FP32 results of the CSC path).
template <typename T>
__global__ __launch_bounds__(256) void finish_y(T *__restrict__ y, const double *__restrict__ acc,
                                                int32_t m, double alpha, double beta) {
  for (int64_t r = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; r < m;
       r += int64_t(gridDim.x) * blockDim.x) {
    const double b = beta == 0.0 ? 0.0 : beta * static_cast<double>(y[r]);
    y[r] = static_cast<T>(alpha * acc[r] + b);
  }
}

// ACC: the array atomically accumulated into (y itself for FP64, else the
// FP64 workspace).  SCALE: alpha is applied per product (FP64 into y) or in
// finish_y (workspace).
template <int VT, int K, typename ACC>
__global__ __launch_bounds__(512) void spmv_csc_scatter(
    const int32_t *__restrict__ col_ptr, const int32_t *__restrict__ row_idx,
    const typename vt_traits<VT>::V *__restrict__ val, const msrep_part *__restrict__ parts,
    const int32_t *__restrict__ lptr, int32_t np, const typename vt_traits<VT>::T *__restrict__ x,
    ACC *__restrict__ acc, int32_t m, int32_t n, double alpha) {
  using Tr = vt_traits<VT>;
  using V = typename Tr::V;
  using Acc = typename Tr::A;
  constexpr int CH = kWave * K;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  (void)col_ptr;

  const int lane = lane_id();
  const int wid = threadIdx.x / kWave;
  const int wpb = blockDim.x / kWave;
  const int p = xcd_block(blockIdx.x, gridDim.x) * wpb + wid;
  if (p >= np) return;
  int32_t *s_col = reinterpret_cast<int32_t *>(lds_raw + wid * csc_lds_per_wave<K>());

  const msrep_part *pp = parts + p;
  const int64_t s0 = uniform(pp->start_idx);
  const int64_t e0 = uniform(pp->end_idx);
  const int32_t c0 = uniform(pp->start_row);  // first column
  const int32_t R = uniform(pp->end_row) - c0 + 1;
  const int32_t *__restrict__ lp = lptr + uniform(pp->lptr_off);
  const int32_t nloc = static_cast<int32_t>(e0 - s0 + 1);
  const int32_t lead = static_cast<int32_t>(s0 % K);
  int32_t j0 = 0;  // local column containing the chunk's first position
  for (int32_t cb = -lead; cb < nloc; cb += CH) {
    const int32_t ce = cb + CH < nloc ? cb + CH : nloc;
    const int32_t q0 = cb + lane * K;
    int32_t rows[K];
    V v[K];
    bool full = q0 >= 0 && q0 + K <= nloc;
    if (full) {
      load_vec<int32_t, K>(row_idx + s0 + q0, rows);
      load_vec<V, K>(val + s0 + q0, v);
    } else {
#pragma unroll
      for (int t = 0; t < K; ++t) {
        const int32_t q = q0 + t;
        rows[t] = -1;
        v[t] = V(0);
        if (q >= 0 && q < nloc) {
          rows[t] = row_idx[s0 + q];
          v[t] = val[s0 + q];
        }
      }
    }
    // columns starting inside the chunk mark their first position
#pragma unroll
    for (int t = 0; t < K; ++t) s_col[lane * K + t] = -1;
    wave_lds_sync();
    int32_t jb = j0, cnt;
    for (;;) {
      const int32_t j = jb + lane;
      const int32_t a = (j >= 0 && j <= R) ? lp[j] : 0x7fffffff;
      const bool in = j <= R - 1 && a < ce;
      if (in && j > j0) {
        const int32_t pos = a - cb;
        if (pos >= 0 && pos < CH) atomicMax(&s_col[pos], j);  // the non-empty column wins
      }
      cnt = __popcll(__ballot(in));
      if (cnt < kWave) break;
      jb += kWave;
    }
    const int32_t j1 = jb + cnt - 1;
    wave_lds_sync();
    int32_t cj[K];
    int32_t mx = j0;
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const int32_t h = s_col[lane * K + t];
      mx = h > mx ? h : mx;
      cj[t] = mx;
    }
    int32_t agg = mx;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int32_t o = shfl_up_i(agg, d);
      if (lane >= d) agg = o > agg ? o : agg;
    }
    int32_t cin = shfl_up_i(agg, 1);
    if (lane == 0) cin = j0;
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const int32_t q = q0 + t;
      const int32_t j = cj[t] > cin ? cj[t] : cin;
      const int32_t c = c0 + j;
      if (q < 0 || q >= nloc) continue;
      if (static_cast<uint32_t>(rows[t]) >= static_cast<uint32_t>(m)) continue;
      if (static_cast<uint32_t>(c) >= static_cast<uint32_t>(n)) continue;
      const Acc pr = Tr::val(v[t]) * static_cast<Acc>(x[c]);
      if constexpr (VT == MSREP_F64) {
        atomicAdd(acc + rows[t], static_cast<ACC>(alpha * static_cast<double>(pr)));
      } else {
        atomicAdd(acc + rows[t], static_cast<ACC>(pr));
      }
    }
    // the column holding the chunk's last position continues, unless it ends
    const int32_t nxt = (j1 + 1 >= 0 && j1 + 1 <= R) ? lp[j1 + 1] : nloc;
    j0 = nxt > ce ? j1 : j1 + 1;
    wave_lds_sync();
  }
}

}  // namespace msrep
