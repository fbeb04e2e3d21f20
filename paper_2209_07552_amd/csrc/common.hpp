// Internal helpers shared by the libmsrep translation units: status/error
// plumbing for the C ABI, argument checks, and small CDNA wave64 device
// utilities.  Nothing here is exported.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <type_traits>

#include "msrep.h"

namespace msrep {

constexpr int kWave = 64;  // CDNA wavefront width
constexpr int kXcds = 8;   // MI355X: 8 accelerator complex dies, one L2 each

// ------------------------------------------------------------ host side
std::string &last_error();
msrep_status fail(msrep_status code, const char *fmt, ...);
inline msrep_status ok() {
  last_error().clear();
  return MSREP_OK;
}

#define MSREP_HIP(call)                                                   \
  do {                                                                    \
    hipError_t e_ = (call);                                               \
    if (e_ != hipSuccess)                                                 \
      return ::msrep::fail(MSREP_ERR_HIP, "%s failed: %s", #call,         \
                           hipGetErrorString(e_));                        \
  } while (0)

#define MSREP_LAUNCHED(what)                                              \
  do {                                                                    \
    hipError_t e_ = hipGetLastError();                                    \
    if (e_ != hipSuccess)                                                 \
      return ::msrep::fail(MSREP_ERR_HIP, "launch of %s failed: %s", what,\
                           hipGetErrorString(e_));                        \
  } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Event pair around one kernel launch while msrep_timing is enabled (no-ops
// otherwise); name must be a string literal.
void timing_begin(const char *name, hipStream_t s);
void timing_end(const char *name, hipStream_t s);

// O(1) descriptor checks shared by every entry point.
msrep_status check_mat(const msrep_mat *A, const char *who);
// Boundary merge of the row-split formats over ncols right-hand sides: column
// j of y (row stride ldy) from the carries at carry + j*cstride.
msrep_status launch_merge_rows(const msrep_mat *A, const msrep_part *parts, int32_t np,
                               const double *carry, void *y, double alpha, double beta,
                               int64_t ldy, int64_t cstride, int ncols, hipStream_t s);
int value_bytes(int32_t vtype);
// x / y element size for a matrix of this value type.
inline int vec_bytes(int32_t vtype) { return vtype == MSREP_F64 ? 8 : 4; }
// Rows of the compressed or sorted dimension (CSR, COO: m; CSC, COO_COL: n).
inline int32_t major_dim(const msrep_mat *A) {
  return A->fmt == MSREP_CSC || A->fmt == MSREP_COO_COL ? A->n : A->m;
}
// Formats whose SpMV runs the bucketed column-merge path (partial vectors
// kept sparse) rather than the row-split path.
inline bool bucketed_fmt(int32_t fmt) {
  return fmt == MSREP_CSC || fmt == MSREP_COO_ANY || fmt == MSREP_COO_COL;
}

__host__ __device__ constexpr size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------- device side
// Raw buffer resources (CDNA "V#"): loads through them are bounds-checked by
// the hardware against num_records bytes and return 0 outside, so every lane
// can issue the same loads with no branch and no out-of-range access.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // gfx9-family raw buffer, 32-bit data format
constexpr int kNt = 2;                  // cache policy bit: non-temporal (streamed once)

// base and bytes must be the same on every lane of the wavefront; they are
// read from the first lane so the descriptor lives in scalar registers.
__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint32_t bytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(a));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(a >> 32));
  void *p = reinterpret_cast<void *>((static_cast<uint64_t>(hi) << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(
      p, 0, static_cast<int>(__builtin_amdgcn_readfirstlane(bytes)), kRsrcWord3);
}

// One element at byte offset `off` (0 when out of range).
template <typename E, int aux = 0>
__device__ __forceinline__ E buf_load(rsrc_t r, uint32_t off) {
  if constexpr (sizeof(E) == 8) {
    const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, aux);
    return __builtin_bit_cast(E, w);
  } else if constexpr (sizeof(E) == 4) {
    return __builtin_bit_cast(E, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, aux));
  } else {
    static_assert(sizeof(E) == 2, "2, 4 or 8 bytes");
    return __builtin_bit_cast(E, __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, aux));
  }
}

// K consecutive elements starting at byte offset `off` (16-byte pieces).
template <typename E, int K, int aux = 0>
__device__ __forceinline__ void buf_load_vec(rsrc_t r, uint32_t off, E (&out)[K]) {
  constexpr int bytes = K * sizeof(E);
  uint32_t *o = reinterpret_cast<uint32_t *>(out);
  if constexpr (bytes % 16 == 0) {
#pragma unroll
    for (int v = 0; v < bytes / 16; ++v) {
      const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16 * v, 0, aux);
      o[4 * v] = w.x;
      o[4 * v + 1] = w.y;
      o[4 * v + 2] = w.z;
      o[4 * v + 3] = w.w;
    }
  } else {
    static_assert(bytes == 8, "8 or a multiple of 16 bytes");
    const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, aux);
    o[0] = w.x;
    o[1] = w.y;
  }
}

// Block index remapped so that each XCD (blocks are dealt to the 8 XCDs
// round-robin by id) receives one contiguous run of logical blocks: its L2
// then sees a contiguous slice of the matrix and of y.
__device__ __forceinline__ int xcd_block(int b, int nblocks) {
  const int q = nblocks / kXcds, r = nblocks % kXcds;
  const int x = b % kXcds, i = b / kXcds;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Wavefronts over np partitions, without atomics: wavefront gw of W takes
// partitions gw, gw + W, gw + 2W, ... (a single one when the grid has a
// wavefront per partition).  The wavefront ids follow the XCD-aware block
// order, so at any moment the resident wavefronts work on one contiguous
// window of partitions and each XCD on a contiguous part of it.
struct PartStride {
  int32_t p, step, np;
  __device__ __forceinline__ PartStride(int32_t np_) : np(np_) {
    const int wpb = blockDim.x / kWave;
    p = xcd_block(blockIdx.x, gridDim.x) * wpb + static_cast<int>(threadIdx.x / kWave);
    step = gridDim.x * wpb;
  }
};

// Keep the compiler from moving LDS accesses of one wavefront across this
// point; a single wavefront's LDS operations execute in program order.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T uniform(T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "uniform: 4 or 8 bytes");
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
  } else {
    const int64_t u = __builtin_bit_cast(int64_t, v);
    const int lo = __builtin_amdgcn_readfirstlane(static_cast<int>(u));
    const int hi = __builtin_amdgcn_readfirstlane(static_cast<int>(u >> 32));
    return __builtin_bit_cast(T, (static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo));
  }
}

// Value of lane `src` (wave-uniform) broadcast to all lanes.
__device__ __forceinline__ int read_lane(int v, int src) {
  return __builtin_amdgcn_readlane(v, src);
}

// Shift up by d lanes within the wavefront (lanes below d get their own value).
__device__ __forceinline__ int shfl_up_i(int v, int d) {
  const int l = lane_id();
  const int src = l >= d ? l - d : l;
  return __builtin_amdgcn_ds_bpermute(src << 2, v);
}
__device__ __forceinline__ float shfl_up_f(float v, int d) {
  return __builtin_bit_cast(float, shfl_up_i(__builtin_bit_cast(int, v), d));
}
__device__ __forceinline__ double shfl_up_d(double v, int d) {
  const int64_t u = __builtin_bit_cast(int64_t, v);
  const int lo = shfl_up_i(static_cast<int>(u), d);
  const int hi = shfl_up_i(static_cast<int>(u >> 32), d);
  return __builtin_bit_cast(double, (static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo));
}
template <typename A>
__device__ __forceinline__ A shfl_up(A v, int d);
template <>
__device__ __forceinline__ float shfl_up<float>(float v, int d) { return shfl_up_f(v, d); }
template <>
__device__ __forceinline__ double shfl_up<double>(double v, int d) { return shfl_up_d(v, d); }

// ------------------------------------------------- DPP wavefront scans
// Lane moves through the data-parallel-primitive path (GCN-style DPP kept by
// CDNA): row_shr:n shifts within rows of 16 lanes, row_bcast:15 / :31 pass a
// row's last lane to the following rows, wave_shr:1 shifts the whole wave.
// Lanes with no source receive 0.
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143, kDppWaveShr1 = 0x138;

template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, dpp_i<CTRL, ROWS>(__builtin_bit_cast(int, v)));
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_d(double v) {
  const int64_t u = __builtin_bit_cast(int64_t, v);
  const int lo = dpp_i<CTRL, ROWS>(static_cast<int>(u));
  const int hi = dpp_i<CTRL, ROWS>(static_cast<int>(u >> 32));
  return __builtin_bit_cast(double, (static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo));
}
template <int CTRL, int ROWS = 0xF, typename A>
__device__ __forceinline__ A dpp(A v) {
  if constexpr (sizeof(A) == 8)
    return dpp_d<CTRL, ROWS>(v);
  else if constexpr (std::is_integral_v<A>)
    return static_cast<A>(dpp_i<CTRL, ROWS>(static_cast<int>(v)));
  else
    return dpp_f<CTRL, ROWS>(v);
}

// One step of a segmented inclusive scan: combine with the (value, flag) a
// DPP move brings from an earlier lane; a lane whose own segment already
// started (flag set) keeps its value.
template <int CTRL, int ROWS, typename A>
__device__ __forceinline__ void seg_step(A &v, int &f) {
  const A pv = dpp<CTRL, ROWS>(v);
  const int pf = dpp_i<CTRL, ROWS>(f);
  if (!f) v += pv;
  f |= pf;
}

// Inclusive segmented scan across the 64 lanes of (value, "a segment starts
// in or before this lane" flag): within rows of 16 by row shifts, then rows
// 1 and 3 from rows 0 and 2, then rows 2 and 3 from row 1.
template <typename A>
__device__ __forceinline__ void wave_seg_scan(A &v, int &f) {
  seg_step<kDppRowShr1, 0xF>(v, f);
  seg_step<kDppRowShr2, 0xF>(v, f);
  seg_step<kDppRowShr4, 0xF>(v, f);
  seg_step<kDppRowShr8, 0xF>(v, f);
  seg_step<kDppRowBcast15, 0xA>(v, f);
  seg_step<kDppRowBcast31, 0xC>(v, f);
}

// Inclusive max-scan across the 64 lanes of non-negative values (lanes with
// no source contribute 0, which never wins).
__device__ __forceinline__ int wave_max_scan_nonneg(int v) {
  int o;
  o = dpp_i<kDppRowShr1, 0xF>(v); v = v > o ? v : o;
  o = dpp_i<kDppRowShr2, 0xF>(v); v = v > o ? v : o;
  o = dpp_i<kDppRowShr4, 0xF>(v); v = v > o ? v : o;
  o = dpp_i<kDppRowShr8, 0xF>(v); v = v > o ? v : o;
  o = dpp_i<kDppRowBcast15, 0xA>(v); v = v > o ? v : o;
  o = dpp_i<kDppRowBcast31, 0xC>(v); v = v > o ? v : o;
  return v;
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
  return __builtin_bit_cast(float, static_cast<uint32_t>(b) << 16);
}

// Knuth's TwoSum on the device (the compensated boundary merge).
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
  const double x = a + b;
  const double z = x - a;
  e = (a - (x - z)) + (b - z);
  s = x;
}

}  // namespace msrep
