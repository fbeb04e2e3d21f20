/*
 * msrep_oracle.c -- plain, slow, obviously correct FP64 CPU oracle for the
 * equal-nnz partitioned sparse matrix-vector product of Chen et al.,
 * "msRep: A Fast yet Light Sparse Matrix Framework for Multi-GPU Systems"
 * (arXiv 2209.07552).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no source with the GPU path.
 *
 * Build: gcc -O2 -fPIC -shared -fopenmp -ffp-contract=off -fno-fast-math
 * (see __init__.py).
 * Contraction is off so that every a*b and a+b below rounds exactly once, as
 * the error-free transformations require; fma() is called explicitly.
 *
 * Contents, each function citing the passage it follows:
 *   - SpMV y = alpha*A*x + beta*y for CSR, CSC and COO storage (Sec. 2.2,
 *     Algorithm 1; CSC swaps the roles of x and y; COO is a single loop over
 *     the nonzeros), every row's dot product accumulated with Dot2 so the
 *     oracle's own error is negligible next to any tolerance.
 *   - The same CSR product in plain FP64 (no compensation) over OpenMP
 *     threads: the row loop a CPU timing baseline runs.
 *   - The same product for k right-hand sides (a row-major block X), every
 *     column as Algorithm 1.
 *   - The partition metadata of pCSR / pCSC / pCOO (Sec. 3.2.1-3.2.3,
 *     Algorithms 2, 4 and 6; pCOO on row-sorted and on column-sorted COO)
 *     including each partition's local row pointer,
 *     and of the paper's equal-rows Baseline split (Sec. 5.3) in the same
 *     records.
 *   - Format conversions between CSR, CSC and row-sorted COO (Sec. 2.1),
 *     and the order that sorts COO given in any order by (row, column) or
 *     (column, row) (Sec. 2.1's COO, sorted as Sec. 3.2.3 takes it).
 *
 * Readings of the paper that this file commits to (the paper is silent,
 * garbled or 1-based in these places):
 *   R1  partitions are numbered i = 0..np-1 (the paper's loop runs 1..np with
 *       floor(i*nnz/np), which would start the last partition at nnz);
 *   R2  end_idx is inclusive, as the "-1" in the paper's formula says;
 *   R3  "BinarySearch(ptr, k)" returns the row containing nonzero k: the
 *       largest r in [0, rows) with ptr[r] <= k (unique, skips empty rows);
 *   R4  the end row's partial status, which the paper says can be inferred
 *       from the next partition, is derived here as end_flag:
 *       end_idx + 1 < ptr[end_row + 1];
 *   R5  the local pointer of a partition with R = end_row - start_row + 1
 *       rows has R + 1 entries lptr[j] = clamp(ptr[start_row + j],
 *       start_idx, end_idx + 1) - start_idx; for 1 <= j < R this is exactly
 *       the paper's loop, and the clamp makes the two ends (0 and the local
 *       nnz) explicit;
 *   R6  i*nnz is formed in 64-bit arithmetic;
 *   R7  an empty partition (np > nnz, or nnz = 0) has end_idx = start_idx - 1,
 *       start_row = (start_idx < nnz ? row containing start_idx : rows),
 *       end_row = start_row - 1, no flags and a one-entry local pointer {0};
 *   R8  a row that no partition covers (empty rows between, before or after
 *       the partitions) is y_r = beta * y_r;
 *   R10 the merge of partial rows is y_r = alpha * (sum of the partial sums)
 *       + beta * y_r with beta applied once per row (the printed merge both
 *       overwrites the earlier partial and applies beta inside the loop);
 *   R11 beta == 0 means y_in is not read (BLAS convention);
 *   R12 pCOO on row-sorted COO takes rows straight from row_idx (the printed
 *       algorithm searches a row_ptr that COO does not have).
 * Storage of the local pointers: partition i's R+1 entries start at
 * lptr_off_i = start_row_i + 2*i, which depends on partition i alone (the
 * paper stresses that every partition can be built independently) and never
 * overlaps partition i+1 because start_row_{i+1} >= end_row_i.  The whole
 * array therefore fits in rows + 2*np entries.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_ERR_ARG (-1)
#define ORACLE_ERR_FORMAT (-2)
#define ORACLE_ERR_SIZE (-3)

/* ------------------------------------------------------------------------ */
/* Error-free transformations (Ogita, Rump, Oishi 2005, "Accurate sum and   */
/* dot product", TwoSum / TwoProduct / Dot2).                               */
/* ------------------------------------------------------------------------ */

/* Knuth's TwoSum: s + e == a + b exactly, s = fl(a + b). */
static void two_sum(double a, double b, double *s, double *e) {
  double x = a + b;
  double z = x - a;
  *e = (a - (x - z)) + (b - z);
  *s = x;
}

/* TwoProduct with a fused multiply-add: p + e == a * b exactly. */
static void two_prod(double a, double b, double *p, double *e) {
  double x = a * b;
  *e = fma(a, b, -x);
  *p = x;
}

/* A Dot2 accumulator: the running sum is hi + lo, as if summed in twice the
 * working precision. */
typedef struct {
  double hi, lo;
} dot2_acc;

static void dot2_add_prod(dot2_acc *acc, double a, double b) {
  double p, pe, s, se;
  two_prod(a, b, &p, &pe);
  two_sum(acc->hi, p, &s, &se);
  acc->hi = s;
  acc->lo = acc->lo + (se + pe);
}

/* y = alpha * dot + beta * y_in, every term again through Dot2, rounded once
 * at the end.  beta == 0 leaves y_in unread (R11). */
static double dot2_finish(const dot2_acc *dot, double alpha, double beta,
                          double y_in) {
  dot2_acc r = {0.0, 0.0};
  dot2_add_prod(&r, alpha, dot->hi);
  dot2_add_prod(&r, alpha, dot->lo);
  if (beta != 0.0) dot2_add_prod(&r, beta, y_in);
  return r.hi + r.lo;
}

/* Tolerance scale of a row: |alpha| * (|A||x|)_i + |beta| * |y_i| (all terms
 * are non-negative, so plain summation is accurate to a relative n*u). */
static double row_scale(double abs_dot, double alpha, double beta,
                        double y_in) {
  double s = fabs(alpha) * abs_dot;
  if (beta != 0.0) s += fabs(beta) * fabs(y_in);
  return s;
}

/* ------------------------------------------------------------------------ */
/* SpMV (Sec. 2.2, Algorithm 1 with reading R10/R11 for beta).              */
/* ------------------------------------------------------------------------ */

/* CSR: row i is the nonzeros row_ptr[i] .. row_ptr[i+1]-1 (Sec. 2.1.2);
 * y_i = alpha * sum_j val_j * x[col_idx_j] + beta * y_i (Algorithm 1). */
int oracle_spmv_csr(int32_t m, int32_t n, const int32_t *row_ptr,
                    const int32_t *col_idx, const double *val, const double *x,
                    double alpha, double beta, const double *y_in,
                    double *y_out, double *scale_out) {
  if (m < 0 || n < 0 || !row_ptr || !y_out) return ORACLE_ERR_ARG;
  for (int64_t i = 0; i < m; ++i) {
    dot2_acc acc = {0.0, 0.0};
    double abs_dot = 0.0;
    for (int64_t j = row_ptr[i]; j < row_ptr[i + 1]; ++j) {
      int32_t c = col_idx[j];
      if (c < 0 || c >= n) return ORACLE_ERR_FORMAT;
      dot2_add_prod(&acc, val[j], x[c]);
      abs_dot += fabs(val[j]) * fabs(x[c]);
    }
    double yi = (beta != 0.0) ? y_in[i] : 0.0;
    y_out[i] = dot2_finish(&acc, alpha, beta, yi);
    if (scale_out) scale_out[i] = row_scale(abs_dot, alpha, beta, yi);
  }
  return ORACLE_OK;
}

/* The same CSR product without compensation: every row's dot product is
 * summed left to right in plain FP64, y_i = alpha * s_i + beta * y_i, rows
 * split over nthreads OpenMP threads in contiguous static blocks (rows are
 * independent, so the result does not depend on nthreads).  This is the
 * plain row loop of Algorithm 1, the CPU baseline a timing is compared with;
 * its rounding error is that of ordinary recursive summation, so it is
 * checked against the Dot2 result above by tolerance only. */
int oracle_spmv_csr_plain(int32_t m, int32_t n, const int32_t *row_ptr,
                          const int32_t *col_idx, const double *val,
                          const double *x, double alpha, double beta,
                          const double *y_in, double *y_out, int32_t nthreads) {
  if (m < 0 || n < 0 || !row_ptr || !y_out || nthreads < 1) return ORACLE_ERR_ARG;
  int bad = 0;
#pragma omp parallel for num_threads(nthreads) schedule(static) reduction(| : bad)
  for (int64_t i = 0; i < m; ++i) {
    double s = 0.0;
    for (int64_t j = row_ptr[i]; j < row_ptr[i + 1]; ++j) {
      int32_t c = col_idx[j];
      if (c < 0 || c >= n) {
        bad = 1;
        break;
      }
      s += val[j] * x[c];
    }
    y_out[i] = (beta != 0.0) ? alpha * s + beta * y_in[i] : alpha * s;
  }
  return bad ? ORACLE_ERR_FORMAT : ORACLE_OK;
}

/* Several right-hand sides (the sparse matrix times several dense vectors
 * that Sec. 2.3 groups with SpMV): Y = alpha*A*X + beta*Y_in for the k columns of the row-major
 * X (n x k, row c at X + c*ldx) and Y (m x k, row i at Y + i*ldy), i.e.
 * Algorithm 1 once per column, each (row, column) dot product kept in its own
 * Dot2 accumulator.  Columns beyond k are not touched.  scale_out (m x k,
 * leading dimension k) may be NULL. */
int oracle_spmm_csr(int32_t m, int32_t n, int32_t k, const int32_t *row_ptr,
                    const int32_t *col_idx, const double *val, const double *X,
                    int64_t ldx, double alpha, double beta, const double *Y_in,
                    int64_t ldy, double *Y_out, double *scale_out) {
  if (m < 0 || n < 0 || k < 0 || !row_ptr || ldx < k || ldy < k) return ORACLE_ERR_ARG;
  if (k == 0 || m == 0) return ORACLE_OK;
  if (!Y_out) return ORACLE_ERR_ARG;
  for (int64_t i = 0; i < m; ++i) {
    for (int64_t t = 0; t < k; ++t) {
      dot2_acc acc = {0.0, 0.0};
      double abs_dot = 0.0;
      for (int64_t j = row_ptr[i]; j < row_ptr[i + 1]; ++j) {
        int32_t c = col_idx[j];
        if (c < 0 || c >= n) return ORACLE_ERR_FORMAT;
        double xv = X[(int64_t)c * ldx + t];
        dot2_add_prod(&acc, val[j], xv);
        abs_dot += fabs(val[j]) * fabs(xv);
      }
      double yi = (beta != 0.0) ? Y_in[i * ldy + t] : 0.0;
      Y_out[i * ldy + t] = dot2_finish(&acc, alpha, beta, yi);
      if (scale_out) scale_out[i * k + t] = row_scale(abs_dot, alpha, beta, yi);
    }
  }
  return ORACLE_OK;
}

/* Shared tail of the CSC and COO oracles, whose loops visit a row's nonzeros
 * out of row order and therefore keep one Dot2 accumulator per row. */
static void finish_rows(int32_t m, const dot2_acc *acc, const double *abs_dot,
                        double alpha, double beta, const double *y_in,
                        double *y_out, double *scale_out) {
  for (int64_t i = 0; i < m; ++i) {
    double yi = (beta != 0.0) ? y_in[i] : 0.0;
    y_out[i] = dot2_finish(&acc[i], alpha, beta, yi);
    if (scale_out) scale_out[i] = row_scale(abs_dot[i], alpha, beta, yi);
  }
}

/* CSC: column j is the nonzeros col_ptr[j] .. col_ptr[j+1]-1 with their row
 * indices (Sec. 2.1.3); the product swaps the roles of x and y (Sec. 2.2):
 * every nonzero of column j adds val * x[j] to y[row_idx]. */
int oracle_spmv_csc(int32_t m, int32_t n, const int32_t *col_ptr,
                    const int32_t *row_idx, const double *val, const double *x,
                    double alpha, double beta, const double *y_in,
                    double *y_out, double *scale_out) {
  if (m < 0 || n < 0 || !col_ptr || !y_out) return ORACLE_ERR_ARG;
  dot2_acc *acc = (dot2_acc *)calloc((size_t)m + 1, sizeof(dot2_acc));
  double *abs_dot = (double *)calloc((size_t)m + 1, sizeof(double));
  if (!acc || !abs_dot) {
    free(acc);
    free(abs_dot);
    return ORACLE_ERR_SIZE;
  }
  int rc = ORACLE_OK;
  for (int64_t j = 0; j < n && rc == ORACLE_OK; ++j) {
    for (int64_t k = col_ptr[j]; k < col_ptr[j + 1]; ++k) {
      int32_t r = row_idx[k];
      if (r < 0 || r >= m) {
        rc = ORACLE_ERR_FORMAT;
        break;
      }
      dot2_add_prod(&acc[r], val[k], x[j]);
      abs_dot[r] += fabs(val[k]) * fabs(x[j]);
    }
  }
  if (rc == ORACLE_OK)
    finish_rows(m, acc, abs_dot, alpha, beta, y_in, y_out, scale_out);
  free(acc);
  free(abs_dot);
  return rc;
}

/* COO: one loop over all nonzeros; nonzero k adds val_k * x[col_idx_k] to
 * y[row_idx_k] (Sec. 2.2).  Any order of the nonzeros is accepted here. */
int oracle_spmv_coo(int32_t m, int32_t n, int64_t nnz, const int32_t *row_idx,
                    const int32_t *col_idx, const double *val, const double *x,
                    double alpha, double beta, const double *y_in,
                    double *y_out, double *scale_out) {
  if (m < 0 || n < 0 || nnz < 0 || !y_out) return ORACLE_ERR_ARG;
  dot2_acc *acc = (dot2_acc *)calloc((size_t)m + 1, sizeof(dot2_acc));
  double *abs_dot = (double *)calloc((size_t)m + 1, sizeof(double));
  if (!acc || !abs_dot) {
    free(acc);
    free(abs_dot);
    return ORACLE_ERR_SIZE;
  }
  int rc = ORACLE_OK;
  for (int64_t k = 0; k < nnz; ++k) {
    int32_t r = row_idx[k], c = col_idx[k];
    if (r < 0 || r >= m || c < 0 || c >= n) {
      rc = ORACLE_ERR_FORMAT;
      break;
    }
    dot2_add_prod(&acc[r], val[k], x[c]);
    abs_dot[r] += fabs(val[k]) * fabs(x[c]);
  }
  if (rc == ORACLE_OK)
    finish_rows(m, acc, abs_dot, alpha, beta, y_in, y_out, scale_out);
  free(acc);
  free(abs_dot);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Partition metadata (Sec. 3.2, Algorithms 2, 4, 6; readings R1-R7, R12).  */
/* ------------------------------------------------------------------------ */

/* R3: the row containing nonzero k, i.e. the largest r in [0, rows) with
 * ptr[r] <= k.  Requires 0 <= k < ptr[rows].  Plain bisection on [lo, hi). */
static int32_t row_containing(const int32_t *ptr, int32_t rows, int64_t k) {
  int32_t lo = 0, hi = rows; /* invariant: ptr[lo] <= k < ptr[hi] */
  while (hi - lo > 1) {
    int32_t mid = lo + (hi - lo) / 2;
    if ((int64_t)ptr[mid] <= k)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

/*
 * Partition a compressed matrix (CSR row_ptr for pCSR, Algorithm 2; CSC
 * col_ptr for pCSC, Algorithm 4 -- identical with rows read as columns) into
 * np equal-nnz partitions.  Outputs are np-long arrays; lptr receives the
 * local pointers at lptr_off (see the header comment), lptr_cap entries
 * available.  *lptr_len gets one past the last entry written.
 */
int oracle_partition_ptr(int32_t rows, const int32_t *ptr, int32_t np,
                         int64_t *start_idx, int64_t *end_idx,
                         int32_t *start_row, int32_t *end_row,
                         int32_t *start_flag, int32_t *end_flag,
                         int64_t *lptr_off, int32_t *lptr, int64_t lptr_cap,
                         int64_t *lptr_len) {
  if (rows < 0 || np <= 0 || !ptr) return ORACLE_ERR_ARG;
  int64_t nnz = ptr[rows];
  int64_t len = 0;
  for (int32_t i = 0; i < np; ++i) {
    int64_t s = ((int64_t)i * nnz) / np;            /* R1, R6 */
    int64_t e = ((int64_t)(i + 1) * nnz) / np - 1;  /* R2 */
    start_idx[i] = s;
    end_idx[i] = e;
    int64_t off = 0;
    if (s > e) { /* R7: empty partition */
      int32_t sr = (s < nnz) ? row_containing(ptr, rows, s) : rows;
      start_row[i] = sr;
      end_row[i] = sr - 1;
      start_flag[i] = 0;
      end_flag[i] = 0;
      off = (int64_t)sr + 2 * (int64_t)i;
      if (off + 1 > lptr_cap) return ORACLE_ERR_SIZE;
      lptr[off] = 0;
      lptr_off[i] = off;
      if (off + 1 > len) len = off + 1;
      continue;
    }
    int32_t sr = row_containing(ptr, rows, s);
    int32_t er = row_containing(ptr, rows, e);
    start_row[i] = sr;
    end_row[i] = er;
    start_flag[i] = (s > ptr[sr]) ? 1 : 0;            /* Algorithm 2 */
    end_flag[i] = (e + 1 < (int64_t)ptr[er + 1]) ? 1 : 0; /* R4 */
    int64_t R = (int64_t)er - sr + 1;
    off = (int64_t)sr + 2 * (int64_t)i;
    if (off + R + 1 > lptr_cap) return ORACLE_ERR_SIZE;
    for (int64_t j = 0; j <= R; ++j) { /* R5 */
      int64_t p = ptr[sr + j];
      if (p < s) p = s;
      if (p > e + 1) p = e + 1;
      lptr[off + j] = (int32_t)(p - s);
    }
    lptr_off[i] = off;
    if (off + R + 1 > len) len = off + R + 1;
  }
  if (lptr_len) *lptr_len = len;
  return ORACLE_OK;
}

/*
 * pCOO on row-sorted COO (Sec. 3.2.3, Algorithm 6 with reading R12): the
 * same equal-nnz split, with the start/end rows read from row_idx.  There is
 * no local pointer; lptr_off is 0 for every partition.
 */
int oracle_partition_coo(int32_t rows, int64_t nnz, const int32_t *row_idx,
                         int32_t np, int64_t *start_idx, int64_t *end_idx,
                         int32_t *start_row, int32_t *end_row,
                         int32_t *start_flag, int32_t *end_flag,
                         int64_t *lptr_off) {
  if (rows < 0 || nnz < 0 || np <= 0) return ORACLE_ERR_ARG;
  for (int64_t k = 1; k < nnz; ++k)
    if (row_idx[k] < row_idx[k - 1]) return ORACLE_ERR_FORMAT;
  for (int32_t i = 0; i < np; ++i) {
    int64_t s = ((int64_t)i * nnz) / np;
    int64_t e = ((int64_t)(i + 1) * nnz) / np - 1;
    start_idx[i] = s;
    end_idx[i] = e;
    lptr_off[i] = 0;
    if (s > e) {
      int32_t sr = (s < nnz) ? row_idx[s] : rows;
      start_row[i] = sr;
      end_row[i] = sr - 1;
      start_flag[i] = 0;
      end_flag[i] = 0;
      continue;
    }
    start_row[i] = row_idx[s];
    end_row[i] = row_idx[e];
    start_flag[i] = (s > 0 && row_idx[s - 1] == row_idx[s]) ? 1 : 0;
    end_flag[i] = (e + 1 < nnz && row_idx[e + 1] == row_idx[e]) ? 1 : 0;
  }
  return ORACLE_OK;
}

/*
 * The paper's Baseline split (Sec. 5.3), the comparison point of the
 * equal-nnz partitions: partition i takes the whole rows (CSC: columns)
 * floor(i*rows/np) .. floor((i+1)*rows/np) - 1 whatever their nonzeros, so
 * no row is split (both flags 0).  The records keep the equal-nnz meaning
 * of every field: start_idx / end_idx are the first and last nonzero of the
 * block, start_row / end_row the rows holding them (R3), the local pointer
 * follows R5 at start_row + 2*i, and a block without nonzeros is an empty
 * partition in the sense of R7.
 */
int oracle_partition_rows_ptr(int32_t rows, const int32_t *ptr, int32_t np,
                              int64_t *start_idx, int64_t *end_idx,
                              int32_t *start_row, int32_t *end_row,
                              int32_t *start_flag, int32_t *end_flag,
                              int64_t *lptr_off, int32_t *lptr, int64_t lptr_cap,
                              int64_t *lptr_len) {
  if (rows < 0 || np <= 0 || !ptr) return ORACLE_ERR_ARG;
  int64_t nnz = ptr[rows];
  int64_t len = 0;
  for (int32_t i = 0; i < np; ++i) {
    int64_t r_lo = ((int64_t)i * rows) / np;
    int64_t r_hi = ((int64_t)(i + 1) * rows) / np; /* one past the block */
    int64_t s = ptr[r_lo];
    int64_t e = (int64_t)ptr[r_hi] - 1;
    int32_t sr = (s < nnz) ? row_containing(ptr, rows, s) : rows;
    int32_t er = (s <= e) ? row_containing(ptr, rows, e) : sr - 1;
    start_idx[i] = s;
    end_idx[i] = e;
    start_row[i] = sr;
    end_row[i] = er;
    start_flag[i] = 0;
    end_flag[i] = 0;
    int64_t off = (int64_t)sr + 2 * (int64_t)i;
    int64_t R = (int64_t)er - sr + 1; /* 0 for an empty block */
    if (off + R + 1 > lptr_cap) return ORACLE_ERR_SIZE;
    if (R == 0) {
      lptr[off] = 0;
    } else {
      for (int64_t j = 0; j <= R; ++j) { /* R5 */
        int64_t p = ptr[sr + j];
        if (p < s) p = s;
        if (p > e + 1) p = e + 1;
        lptr[off + j] = (int32_t)(p - s);
      }
    }
    lptr_off[i] = off;
    if (off + R + 1 > len) len = off + R + 1;
  }
  if (lptr_len) *lptr_len = len;
  return ORACLE_OK;
}

/* The Baseline split of row-sorted COO: the same row blocks, their first
 * and last positions found by scanning row_idx. */
int oracle_partition_rows_coo(int32_t rows, int64_t nnz, const int32_t *row_idx,
                              int32_t np, int64_t *start_idx, int64_t *end_idx,
                              int32_t *start_row, int32_t *end_row,
                              int32_t *start_flag, int32_t *end_flag,
                              int64_t *lptr_off) {
  if (rows < 0 || nnz < 0 || np <= 0) return ORACLE_ERR_ARG;
  for (int64_t k = 1; k < nnz; ++k)
    if (row_idx[k] < row_idx[k - 1]) return ORACLE_ERR_FORMAT;
  for (int32_t i = 0; i < np; ++i) {
    int64_t r_lo = ((int64_t)i * rows) / np;
    int64_t r_hi = ((int64_t)(i + 1) * rows) / np;
    int64_t s = 0, e1 = 0; /* positions of the first row >= r_lo, >= r_hi */
    while (s < nnz && row_idx[s] < r_lo) ++s;
    while (e1 < nnz && row_idx[e1] < r_hi) ++e1;
    start_idx[i] = s;
    end_idx[i] = e1 - 1;
    start_row[i] = (s < nnz) ? row_idx[s] : rows;
    end_row[i] = (s <= e1 - 1) ? row_idx[e1 - 1] : start_row[i] - 1;
    start_flag[i] = 0;
    end_flag[i] = 0;
    lptr_off[i] = 0;
  }
  return ORACLE_OK;
}

/*
 * pCOO on column-sorted COO.  Sec. 3.2.3 lets the nonzeros be sorted by
 * column instead of by row (then the split costs O(np*log(n))), and Sec. 4.3
 * merges such partitions by columns, like pCSC.  The split is Algorithm 6
 * with the roles of rows and columns exchanged: the same equal-nnz position
 * ranges, with start/end *columns* read from col_idx (which must be
 * non-decreasing), start_flag = the first column began in an earlier
 * partition, end_flag = the last column continues into a later one.  The
 * records use the start_row / end_row fields for the columns, as pCSC does.
 * By construction these records equal the pCSC records of the same matrix
 * (Algorithm 4), local pointers aside.
 */
int oracle_partition_coo_col(int32_t cols, int64_t nnz, const int32_t *col_idx,
                             int32_t np, int64_t *start_idx, int64_t *end_idx,
                             int32_t *start_col, int32_t *end_col,
                             int32_t *start_flag, int32_t *end_flag,
                             int64_t *lptr_off) {
  return oracle_partition_coo(cols, nnz, col_idx, np, start_idx, end_idx, start_col,
                              end_col, start_flag, end_flag, lptr_off);
}

/* The Baseline split (Sec. 5.3) of column-sorted COO: equal column blocks,
 * as for CSC. */
int oracle_partition_cols_coo_col(int32_t cols, int64_t nnz, const int32_t *col_idx,
                                  int32_t np, int64_t *start_idx, int64_t *end_idx,
                                  int32_t *start_col, int32_t *end_col,
                                  int32_t *start_flag, int32_t *end_flag,
                                  int64_t *lptr_off) {
  return oracle_partition_rows_coo(cols, nnz, col_idx, np, start_idx, end_idx, start_col,
                                   end_col, start_flag, end_flag, lptr_off);
}

/* ------------------------------------------------------------------------ */
/* Format conversions (Sec. 2.1).                                           */
/* ------------------------------------------------------------------------ */

/* CSR -> COO: nonzero k of row r gets row_idx[k] = r; columns and values keep
 * their order. */
int oracle_csr_to_coo(int32_t m, const int32_t *row_ptr, int32_t *row_idx) {
  if (m < 0 || !row_ptr) return ORACLE_ERR_ARG;
  for (int64_t r = 0; r < m; ++r)
    for (int64_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) row_idx[k] = (int32_t)r;
  return ORACLE_OK;
}

/* Row-sorted COO -> CSR: row_ptr[r] = number of nonzeros in rows < r. */
int oracle_coo_to_csr(int32_t m, int64_t nnz, const int32_t *row_idx,
                      int32_t *row_ptr) {
  if (m < 0 || nnz < 0) return ORACLE_ERR_ARG;
  for (int64_t k = 0; k < nnz; ++k) {
    if (row_idx[k] < 0 || row_idx[k] >= m) return ORACLE_ERR_FORMAT;
    if (k > 0 && row_idx[k] < row_idx[k - 1]) return ORACLE_ERR_FORMAT;
  }
  for (int64_t r = 0; r <= m; ++r) row_ptr[r] = 0;
  for (int64_t k = 0; k < nnz; ++k) row_ptr[row_idx[k] + 1] += 1;
  for (int64_t r = 0; r < m; ++r) row_ptr[r + 1] += row_ptr[r];
  return ORACLE_OK;
}

/*
 * Compressed transpose by a stable counting sort: a CSR matrix (m x n) in,
 * its CSC (= the CSR of its transpose, Sec. 2.1.3) out.  Nonzeros are visited
 * in storage order and appended to their column, so within each column they
 * keep their row order.  Called with the roles swapped it turns CSC into CSR.
 * val/val_out may be NULL; perm (optional) receives, for every output slot,
 * the storage position of the nonzero it came from, so that values of any
 * type can be moved the same way.
 */
int oracle_transpose(int32_t m, int32_t n, const int32_t *row_ptr,
                     const int32_t *col_idx, const double *val,
                     int32_t *col_ptr, int32_t *row_idx, double *val_out,
                     int64_t *perm) {
  if (m < 0 || n < 0 || !row_ptr) return ORACLE_ERR_ARG;
  int64_t nnz = row_ptr[m];
  for (int64_t k = 0; k < nnz; ++k)
    if (col_idx[k] < 0 || col_idx[k] >= n) return ORACLE_ERR_FORMAT;
  int64_t *next = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  if (!next) return ORACLE_ERR_SIZE;
  for (int64_t c = 0; c <= n; ++c) col_ptr[c] = 0;
  for (int64_t k = 0; k < nnz; ++k) col_ptr[col_idx[k] + 1] += 1;
  for (int64_t c = 0; c < n; ++c) col_ptr[c + 1] += col_ptr[c];
  for (int64_t c = 0; c < n; ++c) next[c] = col_ptr[c];
  for (int64_t r = 0; r < m; ++r) {
    for (int64_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) {
      int64_t dst = next[col_idx[k]]++;
      row_idx[dst] = (int32_t)r;
      if (val_out) val_out[dst] = val[k];
      if (perm) perm[dst] = k;
    }
  }
  free(next);
  return ORACLE_OK;
}

/*
 * COO in any order -> sorted COO (Sec. 2.1 stores COO as (row, column,
 * value) triples in any order; Sec. 3.2.3 partitions it sorted by row or by
 * column).  perm[j] = the storage position of the j-th entry in the order
 * sorted by (major, minor), entries equal on both keeping their storage
 * order.  Two stable counting sorts, least significant key first: by minor,
 * then by major.  major in [0, n_major), minor in [0, n_minor).
 */
int oracle_coo_sort(int32_t n_major, int32_t n_minor, int64_t nnz, const int32_t *major,
                    const int32_t *minor, int64_t *perm) {
  if (n_major < 0 || n_minor < 0 || nnz < 0 || (nnz > 0 && (!major || !minor || !perm)))
    return ORACLE_ERR_ARG;
  for (int64_t k = 0; k < nnz; ++k)
    if (major[k] < 0 || major[k] >= n_major || minor[k] < 0 || minor[k] >= n_minor)
      return ORACLE_ERR_FORMAT;
  int64_t *tmp = (int64_t *)malloc(((size_t)nnz + 1) * sizeof(int64_t));
  int64_t *cnt = (int64_t *)calloc((size_t)(n_major > n_minor ? n_major : n_minor) + 1,
                                   sizeof(int64_t));
  if (!tmp || !cnt) {
    free(tmp);
    free(cnt);
    return ORACLE_ERR_SIZE;
  }
  /* pass 1: storage order -> stable by minor (into tmp) */
  for (int64_t k = 0; k < nnz; ++k) cnt[minor[k] + 1] += 1;
  for (int64_t c = 0; c < n_minor; ++c) cnt[c + 1] += cnt[c];
  for (int64_t k = 0; k < nnz; ++k) tmp[cnt[minor[k]]++] = k;
  /* pass 2: that order -> stable by major (into perm) */
  for (int64_t c = 0; c <= n_major; ++c) cnt[c] = 0;
  for (int64_t k = 0; k < nnz; ++k) cnt[major[k] + 1] += 1;
  for (int64_t r = 0; r < n_major; ++r) cnt[r + 1] += cnt[r];
  for (int64_t j = 0; j < nnz; ++j) {
    const int64_t k = tmp[j];
    perm[cnt[major[k]]++] = k;
  }
  free(tmp);
  free(cnt);
  return ORACLE_OK;
}
