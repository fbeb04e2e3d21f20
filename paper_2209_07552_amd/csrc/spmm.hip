// msrep_spmm: Y = alpha*A*X + beta*Y for k right-hand sides over the CSR
// partitions, in passes of at most eight columns (kernel: spmm_csr.hpp), each
// followed by the boundary merge of its columns.
#include "common.hpp"
#include "spmm_csr.hpp"

namespace msrep {

msrep_status spmv_launch(const msrep_mat *A, const msrep_part *parts, const int32_t *lptr,
                         int32_t np, const void *x, void *y, double alpha, double beta, int K,
                         int wpb, int pf, int resident, double *carry, hipStream_t s);

namespace {

int spmm_pass_cols(int32_t left) { return left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1; }

template <int VT, int NR, bool BETA0, int CPL>
msrep_status launch_spmm_pass(const msrep_mat *A, const msrep_part *parts, const int32_t *lptr,
                              int32_t np, const void *X, int64_t ldx, void *Y, int64_t ldy,
                              double alpha, double beta, double *carry, hipStream_t s) {
  using Tr = vt_traits<VT>;
  using T = typename Tr::T;
  const int g = (np + kSpmmWaves - 1) / kSpmmWaves;
  // bytes of Y from this pass's first column to the end of its last row
  const uint32_t ybytes = static_cast<uint32_t>(
      ((static_cast<int64_t>(A->m) - 1) * ldy + NR) * static_cast<int64_t>(sizeof(T)));
  const uint32_t xbytes = static_cast<uint32_t>(
      ((static_cast<int64_t>(A->n > 0 ? A->n : 1) - 1) * ldx + NR) * static_cast<int64_t>(sizeof(T)));
  timing_begin("spmm_csr", s);
  hipLaunchKernelGGL((spmm_csr<VT, NR, BETA0, CPL>), dim3(g), dim3(kSpmmWaves * kWave), 0, s, A->idx,
                     static_cast<const typename Tr::V *>(A->val), parts, lptr, np,
                     static_cast<const T *>(X), ldx, static_cast<T *>(Y), ldy, A->m, alpha, beta,
                     carry, 2 * static_cast<int64_t>(np), xbytes, ybytes);
  MSREP_LAUNCHED("spmm_csr");
  timing_end("spmm_csr", s);
  if (np > 1)
    return launch_merge_rows(A, parts, np, carry, Y, alpha, beta, ldy, 2 * static_cast<int64_t>(np),
                             NR, s);
  return MSREP_OK;
}

template <int VT, bool BETA0>
msrep_status spmm_pass(const msrep_mat *A, const msrep_part *parts, const int32_t *lptr,
                       int32_t np, int nr, const void *X, int64_t ldx, void *Y, int64_t ldy,
                       double alpha, double beta, double *carry, hipStream_t s) {
  // eight columns: two per lane (one 8- or 16-byte X load and Y store per
  // position, four lanes per slot) when X and Y rows keep such pairs aligned
  using T = typename vt_traits<VT>::T;
  const size_t pair = 2 * sizeof(T);
  const bool two = ldx % 2 == 0 && ldy % 2 == 0 && reinterpret_cast<uintptr_t>(X) % pair == 0 &&
                   reinterpret_cast<uintptr_t>(Y) % pair == 0;
  switch (nr) {
    case 8:
      return two ? launch_spmm_pass<VT, 8, BETA0, 2>(A, parts, lptr, np, X, ldx, Y, ldy, alpha, beta, carry, s)
                 : launch_spmm_pass<VT, 8, BETA0, 1>(A, parts, lptr, np, X, ldx, Y, ldy, alpha, beta, carry, s);
    // (four columns: one per lane; two per lane left two lanes per slot and
    // measured slower on the stencil)
    case 4: return launch_spmm_pass<VT, 4, BETA0, 1>(A, parts, lptr, np, X, ldx, Y, ldy, alpha, beta, carry, s);
    case 2: return launch_spmm_pass<VT, 2, BETA0, 1>(A, parts, lptr, np, X, ldx, Y, ldy, alpha, beta, carry, s);
    default: return launch_spmm_pass<VT, 1, BETA0, 1>(A, parts, lptr, np, X, ldx, Y, ldy, alpha, beta, carry, s);
  }
}

template <int VT>
msrep_status spmm_vt(const msrep_mat *A, const msrep_part *parts, const int32_t *lptr, int32_t np,
                     int32_t k, const void *X, int64_t ldx, void *Y, int64_t ldy, double alpha,
                     double beta, double *carry, hipStream_t s) {
  using T = typename vt_traits<VT>::T;
  for (int32_t c0 = 0; c0 < k;) {
    const int nr = spmm_pass_cols(k - c0);
    const T *Xc = static_cast<const T *>(X) + c0;
    T *Yc = static_cast<T *>(Y) + c0;
    const msrep_status st =
        beta == 0.0 ? spmm_pass<VT, true>(A, parts, lptr, np, nr, Xc, ldx, Yc, ldy, alpha, beta, carry, s)
                    : spmm_pass<VT, false>(A, parts, lptr, np, nr, Xc, ldx, Yc, ldy, alpha, beta, carry, s);
    if (st) return st;
    c0 += nr;
  }
  return MSREP_OK;
}

}  // namespace
}  // namespace msrep

using namespace msrep;

extern "C" size_t msrep_spmm_ws_bytes(const msrep_mat *A, int32_t np, int32_t k) {
  if (!A || np <= 0 || k < 0) return 0;
  const int32_t cols = k < kSpmmMaxCols ? (k > 0 ? k : 1) : kSpmmMaxCols;
  return align_up(16 * static_cast<size_t>(np) * static_cast<size_t>(cols), 256);
}

extern "C" msrep_status msrep_spmm(const msrep_mat *A, const msrep_part *parts_d,
                                   const int32_t *lptr_d, int32_t np, int32_t k, const void *X_d,
                                   int64_t ldx, void *Y_d, int64_t ldy, double alpha, double beta,
                                   void *ws_d, size_t ws_bytes, void *stream) {
  const char *who = "msrep_spmm";
  if (msrep_status st = check_mat(A, who)) return st;
  if (A->fmt != MSREP_CSR)
    return fail(MSREP_ERR_UNSUPPORTED, "%s: several right-hand sides are taken in CSR only", who);
  if (np <= 0) return fail(MSREP_ERR_ARG, "%s: np must be positive (got %d)", who, np);
  if (k < 0) return fail(MSREP_ERR_ARG, "%s: k must be >= 0 (got %d)", who, k);
  if (!parts_d || !lptr_d) return fail(MSREP_ERR_ARG, "%s: parts_d or lptr_d is NULL", who);
  if (ldx < k || ldy < k)
    return fail(MSREP_ERR_ARG, "%s: ldx (%lld) and ldy (%lld) must be >= k (%d)", who,
                static_cast<long long>(ldx), static_cast<long long>(ldy), k);
  if (k == 0 || A->m == 0) return ok();
  if (!Y_d) return fail(MSREP_ERR_ARG, "%s: Y_d is NULL", who);
  if (A->nnz > 0 && !X_d) return fail(MSREP_ERR_ARG, "%s: X_d is NULL", who);
  if ((static_cast<uint64_t>(A->m) + 1) * 4 >= (uint64_t(1) << 32))
    return fail(MSREP_ERR_UNSUPPORTED, "%s: too many rows", who);
  // X and Y are addressed through 32-bit buffer offsets
  if (static_cast<uint64_t>(A->m) * static_cast<uint64_t>(ldy) * vec_bytes(A->vtype) >=
          (uint64_t(1) << 32) - 512 ||
      static_cast<uint64_t>(A->n) * static_cast<uint64_t>(ldx) * vec_bytes(A->vtype) >=
          (uint64_t(1) << 32) - 512)
    return fail(MSREP_ERR_UNSUPPORTED, "%s: X (n x ldx) or Y (m x ldy) of 4 GiB or more", who);
  const size_t need = msrep_spmm_ws_bytes(A, np, k);
  if (!ws_d || ws_bytes < need)
    return fail(MSREP_ERR_SIZE, "%s: workspace of %zu bytes needed (got %zu)", who, need,
                ws_d ? ws_bytes : size_t(0));
  double *carry = static_cast<double *>(ws_d);
  const hipStream_t s = as_stream(stream);
  // one contiguous column: the single-vector kernel (four nonzeros per lane)
  // is the faster one; its workspace is the same two slots per partition
  if (k == 1 && ldx == 1 && ldy == 1) {
    if (msrep_status st = spmv_launch(A, parts_d, lptr_d, np, X_d, Y_d, alpha, beta, 4, 4, 2, 0,
                                      carry, s))
      return st;
    return ok();
  }
  msrep_status st;
  switch (A->vtype) {
    case MSREP_F64: st = spmm_vt<MSREP_F64>(A, parts_d, lptr_d, np, k, X_d, ldx, Y_d, ldy, alpha, beta, carry, s); break;
    case MSREP_F32: st = spmm_vt<MSREP_F32>(A, parts_d, lptr_d, np, k, X_d, ldx, Y_d, ldy, alpha, beta, carry, s); break;
    default: st = spmm_vt<MSREP_BF16>(A, parts_d, lptr_d, np, k, X_d, ldx, Y_d, ldy, alpha, beta, carry, s); break;
  }
  if (st) return st;
  return ok();
}
