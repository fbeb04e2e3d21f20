// Device-wide scans shared by the conversion and the CSC paths: a reduce
// pass over tiles of kTile elements, one block scanning the tile aggregates,
// and a down-sweep that writes inclusive or exclusive prefixes.
#pragma once

#include "common.hpp"

// Internal linkage: each translation unit that launches these kernels owns
// its own instantiations.
namespace msrep {
namespace {
namespace scan {

constexpr int kBlock = 256;
constexpr int kItems = 16;
constexpr int kTile = kBlock * kItems;  // 4096 elements per block

int64_t tiles(int64_t n) { return (n + kTile - 1) / kTile; }

// ------------------------------------------------------------ scans
struct SumOp {
  template <typename T>
  __device__ static T id() { return T(0); }
  template <typename T>
  __device__ static T op(T a, T b) { return a + b; }
};
struct MaxOp {
  template <typename T>
  __device__ static T id() { return T(-1); }
  template <typename T>
  __device__ static T op(T a, T b) { return a > b ? a : b; }
};

template <typename T, typename Op>
__device__ T block_reduce(T v, T *sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int d = 32; d > 0; d >>= 1) v = Op::template op<T>(v, __shfl_xor(v, d));
  if (lane == 0) sh[w] = v;
  __syncthreads();
  T r = Op::template id<T>();
  for (int i = 0; i < kBlock / 64; ++i) r = Op::template op<T>(r, sh[i]);
  __syncthreads();
  return r;
}

// Exclusive block scan of one value per thread; returns the block total.
template <typename T, typename Op>
__device__ T block_exscan(T v, T &excl, T *sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  T inc = v;
  for (int d = 1; d < 64; d <<= 1) {
    const T o = __shfl_up(inc, d);
    if (lane >= d) inc = Op::template op<T>(o, inc);
  }
  if (lane == 63) sh[w] = inc;
  __syncthreads();
  T before = Op::template id<T>(), total = Op::template id<T>();
  for (int i = 0; i < kBlock / 64; ++i) {
    if (i < w) before = Op::template op<T>(before, sh[i]);
    total = Op::template op<T>(total, sh[i]);
  }
  const T up = __shfl_up(inc, 1);
  excl = Op::template op<T>(before, lane == 0 ? Op::template id<T>() : up);
  __syncthreads();
  return total;
}

template <typename T, typename Op>
__global__ __launch_bounds__(kBlock) void scan_reduce(const T *__restrict__ in, int64_t n,
                                                      T *__restrict__ agg) {
  __shared__ T sh[kBlock / 64];
  const int64_t base = blockIdx.x * int64_t(kTile) + threadIdx.x * int64_t(kItems);
  T v = Op::template id<T>();
#pragma unroll
  for (int i = 0; i < kItems; ++i)
    if (base + i < n) v = Op::template op<T>(v, in[base + i]);
  v = block_reduce<T, Op>(v, sh);
  if (threadIdx.x == 0) agg[blockIdx.x] = v;
}

// Exclusive scan of the nb block aggregates in place (one block, looping).
template <typename T, typename Op>
__global__ __launch_bounds__(kBlock) void scan_aggs(T *__restrict__ agg, int64_t nb) {
  __shared__ T sh[kBlock / 64];
  T carry = Op::template id<T>();
  for (int64_t b0 = 0; b0 < nb; b0 += kBlock) {
    const int64_t i = b0 + threadIdx.x;
    const T v = i < nb ? agg[i] : Op::template id<T>();
    T ex;
    const T tot = block_exscan<T, Op>(v, ex, sh);
    if (i < nb) agg[i] = Op::template op<T>(carry, ex);
    carry = Op::template op<T>(carry, tot);
  }
}

// out = inclusive (or exclusive) scan of in, given the exclusive block
// prefixes; in and out may alias.
template <typename T, typename Op>
__global__ __launch_bounds__(kBlock) void scan_down(const T *in, T *out, int64_t n,
                                                    const T *__restrict__ pre, bool inclusive) {
  __shared__ T sh[kBlock / 64];
  const int64_t base = blockIdx.x * int64_t(kTile) + threadIdx.x * int64_t(kItems);
  T v[kItems];
  T local = Op::template id<T>();
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    v[i] = base + i < n ? in[base + i] : Op::template id<T>();
    local = Op::template op<T>(local, v[i]);
  }
  T ex;
  block_exscan<T, Op>(local, ex, sh);
  T run = Op::template op<T>(pre[blockIdx.x], ex);
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const T next = Op::template op<T>(run, v[i]);
    if (base + i < n) out[base + i] = inclusive ? next : run;
    run = next;
  }
}

template <typename T, typename Op>
msrep_status device_scan(const T *in, T *out, int64_t n, T *agg, bool inclusive, hipStream_t s) {
  if (n <= 0) return MSREP_OK;
  const int64_t nb = tiles(n);
  hipLaunchKernelGGL((scan_reduce<T, Op>), dim3(nb), dim3(kBlock), 0, s, in, n, agg);
  MSREP_LAUNCHED("scan_reduce");
  hipLaunchKernelGGL((scan_aggs<T, Op>), dim3(1), dim3(kBlock), 0, s, agg, nb);
  MSREP_LAUNCHED("scan_aggs");
  hipLaunchKernelGGL((scan_down<T, Op>), dim3(nb), dim3(kBlock), 0, s, in, out, n, agg, inclusive);
  MSREP_LAUNCHED("scan_down");
  return MSREP_OK;
}

}  // namespace scan
}  // namespace
}  // namespace msrep
