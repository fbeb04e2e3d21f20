/*
 * msrep.h -- C ABI of libmsrep, an MI355X (gfx950) implementation of the
 * equal-nnz partitioned sparse matrix-vector product of Chen et al., "msRep:
 * A Fast yet Light Sparse Matrix Framework for Multi-GPU Systems" (arXiv
 * 2209.07552), with the paper's split taken across one GPU's compute units,
 * workgroups and wavefronts instead of across GPUs.
 *
 * General conventions
 *   - Every pointer named *_d, and every array inside msrep_mat / msrep_part,
 *     is device memory (HBM of the current HIP device) owned by the caller.
 *     The library never frees caller memory.  Host pointers are marked.
 *   - Streams are hipStream_t passed as void* (NULL = the default stream).
 *     All work is stream-ordered; no call synchronises the device unless its
 *     comment says so.
 *   - Calls return an msrep_status; on failure nothing has been launched and
 *     msrep_last_error() returns a description (thread-local).  No C++
 *     exception crosses this boundary.
 *   - Indices are int32; nonzero positions and offsets are int64.  A matrix
 *     holds fewer than 2^31 nonzeros.
 *   - Cheap O(1) argument checks always run.  The O(nnz) structure checks
 *     (monotone pointers, indices in range, row-sorted COO) run only in
 *     msrep_validate; kernels never read or write outside the arrays the
 *     descriptors give, whatever the contents, but results on invalid
 *     structure are unspecified.
 */
#ifndef MSREP_H
#define MSREP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
typedef int32_t msrep_status;
#define MSREP_OK 0
#define MSREP_ERR_ARG (-1)         /* null pointer, negative size, np <= 0, bad enum */
#define MSREP_ERR_FORMAT (-2)      /* structure invalid (from msrep_validate)        */
#define MSREP_ERR_SIZE (-3)        /* nnz >= 2^31, buffer or workspace too small     */
#define MSREP_ERR_HIP (-4)         /* a HIP runtime call failed                      */
#define MSREP_ERR_BUDGET (-5)      /* a serving request can never fit the budget     */
#define MSREP_ERR_BUSY (-6)        /* serving queue full                             */
#define MSREP_ERR_UNSUPPORTED (-7) /* combination not implemented                    */

/* Text of the last failure on this thread ("" after a success). */
const char *msrep_last_error(void);

/* ------------------------------------------------------------ kernel timing */
/* A profiling aid for measuring single kernels of a call.  While enabled,
 * every kernel msrep_spmv launches (the per-format SpMV kernel, the boundary
 * merge, and the count, scan, scatter, plan, reduce and merge kernels of the
 * CSC path) is bracketed by two HIP events recorded on the caller's stream.
 * msrep_timing_read totals the event-measured durations by kernel name.
 * Process-wide state, off by default; not meant for concurrent callers. */
typedef struct msrep_kernel_time {
  char name[48];   /* kernel name, e.g. "spmv_csr_seg", "csc_scatter"  */
  int64_t calls;   /* launches timed since the last read               */
  double total_ms; /* sum of their durations                           */
} msrep_kernel_time; /* 64 bytes */

/* Enable (nonzero) or disable timing; either way discards what was
 * recorded.  Waits for recorded events that are still pending. */
msrep_status msrep_timing(int32_t enable);

/* Restrict timing to the kernel of this name (NULL or "" = every kernel).
 * Each event record adds a gap of a few microseconds before the next
 * kernel, so timing one kernel perturbs a call far less than timing all. */
msrep_status msrep_timing_only(const char *kernel);

/* Waits for the recorded events, writes up to cap entries (one per kernel
 * name, in order of first launch) and discards the records.  Returns the
 * number of distinct kernels (entries past cap are dropped), or a negative
 * status (MSREP_ERR_ARG for cap < 0 or a NULL out with cap > 0,
 * MSREP_ERR_HIP when an event cannot be read). */
int32_t msrep_timing_read(msrep_kernel_time *out, int32_t cap);

/* A calibration aid, not part of the method: the HBM rate this GPU reaches
 * on plain streams, as the practical ceiling beside the 8 TB/s peak for the
 * SpMV kernels, which stream their index and value arrays.  mode 0 reads
 * `bytes` from src (16-byte loads, one pass; dst receives at most 16 bytes,
 * only if the data hashes to a fixed value), mode 1 copies src to dst.
 * Both buffers are device memory, 16-byte aligned, bytes a multiple of 16
 * (dst at least 16 bytes in mode 0, `bytes` in mode 1, not overlapping src).
 * blocks = workgroups of 256 lanes (0: 65536).  Asynchronous on `stream`.
 * MSREP_ERR_ARG for NULL or misaligned buffers, a bad size or mode. */
msrep_status msrep_probe_stream(const void *src, void *dst, size_t bytes, int32_t mode,
                                int32_t blocks, void *stream);

/* ------------------------------------------------------------ matrices */
/* Storage formats of Sec. 2.1: CSR, CSC (the CSR of the transpose), COO
 * sorted by row (the order Sec. 3.2.3 assumes for pCOO), COO in any order
 * (MSREP_COO_ANY, the variant Sec. 3.2.3 mentions whose partitions need the
 * column-style merge of partial vectors) and COO sorted by column
 * (MSREP_COO_COL: Sec. 3.2.3's other sorted order, split in O(np log n) and
 * merged by columns like pCSC, Sec. 4.3). */
enum { MSREP_CSR = 0, MSREP_CSC = 1, MSREP_COO = 2, MSREP_COO_ANY = 3, MSREP_COO_COL = 4 };

/* Stored value type.  F64 values use FP64 x and y and FP64 arithmetic.  F32
 * and BF16 values use FP32 x and y, FP32 products and in-chunk sums, and FP64
 * for sums carried across chunks and partitions (the boundary merge). */
enum { MSREP_F64 = 0, MSREP_F32 = 1, MSREP_BF16 = 2 };

typedef struct msrep_mat {
  int32_t fmt;   /* MSREP_CSR / MSREP_CSC / MSREP_COO / MSREP_COO_ANY /        */
                 /* MSREP_COO_COL                                               */
  int32_t vtype; /* MSREP_F64 / MSREP_F32 / MSREP_BF16                          */
  int32_t m, n;  /* rows, columns                                               */
  int64_t nnz;   /* number of stored nonzeros                                   */
  const int32_t *ptr;  /* CSR row_ptr[m+1] | CSC col_ptr[n+1] | COO*: NULL     */
  const int32_t *idx;  /* CSR col_idx | CSC row_idx | COO row_idx (sorted) |   */
                       /* COO_ANY row_idx (any order) | COO_COL row_idx       */
  const int32_t *idx2; /* COO, COO_ANY col_idx | COO_COL col_idx (sorted) |     */
                       /* otherwise NULL                                        */
  const void *val;     /* nnz values of vtype (BF16: raw 16-bit patterns)       */
} msrep_mat;

/* Bytes of one stored value of vtype, 0 for an unknown vtype. */
int32_t msrep_vtype_bytes(int32_t vtype);

/* O(nnz) structure check on the GPU: pointer starts at 0, is non-decreasing
 * and ends at nnz; indices in range; COO row indices non-decreasing, COO_COL
 * column indices non-decreasing (no order required for COO_ANY).
 * Returns MSREP_OK or MSREP_ERR_FORMAT (with the first offence described).
 * Synchronises the stream. */
msrep_status msrep_validate(const msrep_mat *A, void *stream);

/* ----------------------------------------------------------- partitions */
/*
 * One partition of pCSR / pCSC / pCOO (Sec. 3.2.1-3.2.3): the nonzeros
 * start_idx .. end_idx (inclusive) of the matrix's storage order.  For CSC
 * the *_row fields hold columns.
 *   start_idx = floor(i*nnz/np), end_idx = floor((i+1)*nnz/np) - 1
 *     (Algorithm 2, partitions numbered from 0, products in 64-bit);
 *   start_row / end_row = the row containing start_idx / end_idx (largest r
 *     with ptr[r] <= k);
 *   start_flag = the first row began in an earlier partition (Algorithm 2);
 *   end_flag   = the last row continues into a later partition (the paper
 *     infers this from the next partition; it is stored for the kernels);
 *   lptr_off   = where this partition's local pointer starts in the lptr
 *     array: start_row + 2*i (0 for pCOO, which has none).
 * Local pointer: R = end_row - start_row + 1 rows, R + 1 entries
 *   lptr[lptr_off + j] = clamp(ptr[start_row + j], start_idx, end_idx + 1)
 *                        - start_idx,  j = 0..R
 * (the paper's local row_ptr with both ends made explicit).  An empty
 * partition (np > nnz) has end_idx = start_idx - 1, start_row = the row of
 * start_idx (or m if start_idx == nnz), end_row = start_row - 1, both flags 0
 * and the single entry lptr[lptr_off] = 0.  COO_COL: the same records with
 * columns in place of rows (start_row / end_row hold the columns of
 * start_idx / end_idx, the flags mark split columns; Algorithm 6 applied to
 * the column index, equal to pCSC's records of the same matrix), no local
 * pointer, lptr_off 0.  COO_ANY: only start_idx and
 * end_idx are defined (equal-nnz position ranges; rows are not grouped):
 * start_row 0, end_row -1, flags 0, lptr_off 0.
 */
typedef struct msrep_part {
  int64_t start_idx, end_idx;
  int32_t start_row, end_row;
  int32_t start_flag, end_flag;
  int64_t lptr_off;
} msrep_part;

/* Entries the lptr array needs for a pCSR (rows = m) or pCSC (rows = n) of np
 * partitions: rows + 2*np.  -1 if an argument is negative or np <= 0. */
int64_t msrep_lptr_bound(int32_t rows, int32_t np);

/*
 * Build np equal-nnz partitions of A on the GPU (Algorithms 2, 4, 6; the
 * local pointers are computed by a device kernel as in the paper's optimised
 * variant, Sec. 4.1).  O(np * log(m) + m) work, every partition independent.
 *   parts_d   : np msrep_part, written.
 *   lptr_d    : lptr_cap int32, written at each partition's entries (gaps
 *               between partitions are left untouched); may be NULL with
 *               lptr_cap 0 for COO.  lptr_cap must be >= msrep_lptr_bound.
 *   lptr_len_d: optional (device int64), receives one past the last entry.
 * COO must be sorted by row; row indices are read at 2*np positions only.
 * COO_COL must be sorted by column; column indices are read at 2*np
 * positions only.
 * COO_ANY reads no indices.
 */
msrep_status msrep_build_partition(const msrep_mat *A, int32_t np,
                                   msrep_part *parts_d, int32_t *lptr_d,
                                   int64_t lptr_cap, int64_t *lptr_len_d,
                                   void *stream);

/*
 * The paper's Baseline split (Sec. 5.3), for comparison with the equal-nnz
 * partitions: partition i holds the whole rows (CSC: columns)
 * floor(i*rows/np) .. floor((i+1)*rows/np) - 1, however many nonzeros they
 * have, so partitions are unequal in work and no row is split.  The records
 * have the meaning given above (start_idx / end_idx the block's first and
 * last nonzero, start_row / end_row the rows holding them, both flags 0,
 * local pointers at start_row + 2*i); a block without nonzeros is an empty
 * partition.  Same arguments, sizes and errors as msrep_build_partition,
 * and every SpMV entry point takes the result like an equal-nnz partition.
 * COO in any order has no row blocks (MSREP_ERR_UNSUPPORTED).  Row-sorted
 * COO is searched by bisection at 2*np positions.
 */
msrep_status msrep_build_partition_rows(const msrep_mat *A, int32_t np,
                                        msrep_part *parts_d, int32_t *lptr_d,
                                        int64_t lptr_cap, int64_t *lptr_len_d,
                                        void *stream);

/* ---------------------------------------------------------- conversion */
/* Workspace bytes msrep_convert needs to turn src into format dst_fmt. */
size_t msrep_convert_ws_bytes(const msrep_mat *src, int32_t dst_fmt);

/*
 * Convert between CSR, CSC, row-sorted COO and column-sorted COO (Sec. 2.1;
 * CSC(A) = CSR(A^T)).  dst->fmt selects the target; dst->m, n, nnz, vtype
 * must equal src's and its arrays must be allocated (CSR: ptr m+1, idx nnz;
 * CSC: ptr n+1, idx nnz; COO, COO_COL: idx nnz, idx2 nnz; val nnz).  Values are moved, never rounded.  Conversions
 * are stable: entries that tie on the new major index keep their storage
 * order, so canonical input (sorted minor indices, no duplicates) gives the
 * unique canonical output.  COO in any order (COO_ANY) may be the source:
 * its entries are sorted stably by the target's major index, ties by its
 * minor index, so equal (row, column) pairs keep their storage order; it is
 * not a target (MSREP_ERR_UNSUPPORTED; msrep_spmv takes it as it is).
 * dst's arrays must not overlap src's: between the passes of its sort a
 * transposing conversion keeps entries in dst's index and value arrays.
 * ws_d: msrep_convert_ws_bytes bytes of device memory.
 */
msrep_status msrep_convert(const msrep_mat *src, msrep_mat *dst, void *ws_d,
                           size_t ws_bytes, void *stream);

/* ----------------------------------------------------------------- SpMV */
/* Launch shape.  A zeroed struct (or NULL) selects the defaults. */
typedef struct msrep_tune {
  int32_t k_per_lane;   /* nonzeros per lane per chunk: 4 (default) or 8       */
  int32_t waves_per_wg; /* wavefronts per workgroup, 1..8 (default 4)          */
  int32_t resident;     /* CSR, COO: 0 (default) one wavefront per partition,  */
                        /* launched as the hardware frees slots; 1: as many    */
                        /* wavefronts as the device holds at once, each taking */
                        /* every W-th partition (W = their number)             */
  int32_t nnz_per_wave; /* partition size the autotuner recommends, so that    */
                        /* np = ceil(nnz / nnz_per_wave); not read by msrep_spmv */
  int32_t pipeline;     /* CSR: chunks of indices/values loaded ahead, 1 or 2  */
                        /* (2 also gathers x one chunk ahead); 0 = default 2.  */
                        /* CSC, COO_COL, COO_ANY (column merge): 1 = one       */
                        /* record per product (value and 32-bit row offset:    */
                        /* one store each, for rows that scatter widely), 2    */
                        /* (default) = values and 16-bit row offsets in two    */
                        /* arrays (2 bytes less), 3 = row windows: each run of */
                        /* partitions sums its products in LDS over the 256-   */
                        /* row windows its rows touch (for banded matrices;    */
                        /* rows outside 30 windows take device atomics).       */
  int32_t _pad;
} msrep_tune;

/* Workspace bytes msrep_spmv needs for A split into np partitions.
 *   CSR, COO: two FP64 partial sums per partition for the boundary merge
 *     (16*np, rounded up to 256).
 *   CSC, COO_ANY, COO_COL: bucket counters (buckets x producers int32), per-bucket piece
 *     tables, one product per nonzero (8 bytes for F64 values, 4 otherwise)
 *     with its row offset (room for either product layout, see
 *     msrep_tune.pipeline), and the partial row arrays of buckets cut into
 *     several pieces: about (s_p + 4)*nnz bytes; the row-window layout's
 *     window lists, contributor lists, window sums and spill sums (8*m
 *     bytes), its sums sharing the products' space.
 *   Matrices of these formats with more than 2^26 rows (more than the
 *   buckets cover) need only the row-window layout.
 * Returns 0 for a malformed descriptor. */
size_t msrep_spmv_ws_bytes(const msrep_mat *A, int32_t np);

/*
 * y = alpha*A*x + beta*y over the np partitions built by msrep_build_partition
 * (Algorithms 3, 5, 7).
 *   CSR, COO: one wavefront streams each partition's nonzeros; rows inside a
 *     partition are written directly; a row split between partitions is
 *     merged by a segmented sum of its partial sums over the partitions
 *     (FP64, TwoSum-compensated) and applying beta once; rows covered by no
 *     partition get beta*y.  Deterministic for a given np and tune.
 *   CSC: the partitions' partial vectors (Algorithm 5, Sec. 4.3 column
 *     merge) are kept sparse: every product is written once, grouped by row
 *     bucket, and each bucket is summed in LDS; no atomics on y.  The order
 *     of the sums within a bucket varies between runs.
 *   COO_ANY, COO_COL: the same bucketed path, each nonzero's column read
 *     from idx2 (lptr_d is not read and may be NULL).  For COO_COL this is
 *     the column-based merge of Sec. 4.3: each partition's partial vector
 *     over y, kept sparse as for CSC.
 *   These three formats take the row-window path (msrep_tune.pipeline 3)
 *   when the tune asks for it, and always when A has more than 2^26 rows
 *   (the bucketed path's limit): its window sums cover the rows each run of
 *   partitions touches most, device atomics the rest, so any row count runs.
 *   x_d: n values, y_d: m values (FP64 for F64 matrices, FP32 otherwise).
 *   beta == 0: y is not read.
 *   ws_d: msrep_spmv_ws_bytes(A, np) bytes, caller-owned, contents free.
 *   tune: NULL for the defaults (see msrep_tune).
 * The call only launches kernels on the stream (no allocation, memset or
 * host synchronisation), so it can be captured into a graph; capture after
 * one uncaptured call with the same launch shape, which fills host-side
 * caches.  Errors: MSREP_ERR_ARG (NULL arrays, np <= 0, bad tune),
 * MSREP_ERR_SIZE (workspace too small), MSREP_ERR_UNSUPPORTED (x or y over
 * 4 GiB), MSREP_ERR_HIP (a launch failed).
 */
msrep_status msrep_spmv(const msrep_mat *A, const msrep_part *parts_d,
                        const int32_t *lptr_d, int32_t np, const void *x_d,
                        void *y_d, double alpha, double beta,
                        const msrep_tune *tune, void *ws_d, size_t ws_bytes,
                        void *stream);

/*
 * msrep_spmv in two parts, for a matrix multiplied many times with the same
 * partitions (an inspector / executor split of Algorithm 5's CSC path).
 * msrep_spmv_prepare runs the structure-only kernels, which read A's indices
 * and the partitions but neither x nor the values: for CSC, the count of
 * every producer's nonzeros per row bucket, their scan into run offsets and
 * the bucket pieces, written to the front of ws_d; for CSR and COO it does
 * nothing.  msrep_spmv_prepared then computes y = alpha*A*x + beta*y like
 * msrep_spmv, using that part of ws_d instead of recomputing it.
 *   Same arguments, checks and errors as msrep_spmv.  ws_d of
 *   msrep_spmv_ws_bytes(A, np) bytes must hold what msrep_spmv_prepare wrote
 *   for the same A structure (m, n, nnz, indices), parts_d and np; calls of
 *   msrep_spmv_prepared leave it intact, a call of msrep_spmv on the same
 *   workspace rewrites it the same way.  Preparing once and calling
 *   msrep_spmv_prepared gives the same y as msrep_spmv up to the order of
 *   the sums within a CSC bucket.  Both only launch kernels on the stream.
 */
msrep_status msrep_spmv_prepare(const msrep_mat *A, const msrep_part *parts_d,
                                const int32_t *lptr_d, int32_t np, void *ws_d,
                                size_t ws_bytes, void *stream);
msrep_status msrep_spmv_prepared(const msrep_mat *A, const msrep_part *parts_d,
                                 const int32_t *lptr_d, int32_t np, const void *x_d,
                                 void *y_d, double alpha, double beta,
                                 const msrep_tune *tune, void *ws_d, size_t ws_bytes,
                                 void *stream);

/*
 * msrep_spmv without a workspace argument, for callers that cannot allocate
 * device memory (code under graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  CSR and row-sorted COO only (others:
 * MSREP_ERR_UNSUPPORTED).  The two FP64 boundary carries per partition live
 * in a static device array of msrep_spmv_noalloc_max_parts() partitions
 * (2^19, 8 MiB), which each GPU the library runs on holds until the process
 * ends; np above that is MSREP_ERR_SIZE.  No allocation, free or memset is
 * made: the carries need no clearing, since a slot's value is used only after the
 * same call's SpMV kernel has written it.  Arguments, kernels, results and
 * other errors are those of msrep_spmv with the same tune (bit-identical y).
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (concurrent streams or host threads) race and must be ordered by the
 * caller.  The first call on a device looks up its copy's address
 * (MSREP_ERR_HIP if that fails).
 */
int32_t msrep_spmv_noalloc_max_parts(void);
msrep_status msrep_spmv_noalloc(const msrep_mat *A, const msrep_part *parts_d,
                                const int32_t *lptr_d, int32_t np, const void *x_d,
                                void *y_d, double alpha, double beta,
                                const msrep_tune *tune, void *stream);

/* Launch shape and partition size for A, picked by timing every candidate on
 * the stream and keeping the fastest median of three runs:
 *   nnz_per_wave in {256, 512, 1024, 2048, 4096} (the equal-nnz np follows),
 *   k_per_lane in {4, 8}, waves_per_wg in {2, 4, 8} (CSR, COO),
 *   pipeline in {1, 2} (CSR), {1, 2, 3} (CSC, COO_COL, COO_ANY),
 *   resident in {0, 1} (CSR, COO).
 * x_d holds n values for the timed SpMVs.  Synchronises the stream.
 * ws_d: at least msrep_autotune_ws_bytes(A) bytes (partitions, local
 * pointers, a y and the SpMV workspace of the largest np). */
size_t msrep_autotune_ws_bytes(const msrep_mat *A);
msrep_status msrep_autotune(const msrep_mat *A, const void *x_d, void *ws_d,
                            size_t ws_bytes, msrep_tune *out, void *stream);

/* --------------------------------------------- several right-hand sides */
/*
 * Y = alpha*A*X + beta*Y for k right-hand sides at once (the sparse matrix
 * times several dense vectors that Sec. 2.3 groups with SpMV): the same
 * equal-nnz CSR partitions and boundary merge as msrep_spmv (Algorithm 3,
 * Sec. 4.3), applied to every column.  A is read once per pass of up to
 * eight columns instead of once per column.
 *   A: CSR only (others: MSREP_ERR_UNSUPPORTED); parts_d, lptr_d, np as
 *   built by msrep_build_partition for A.
 *   X_d: n x k, row-major, leading dimension ldx >= k elements (row i at
 *   X_d + i*ldx); Y_d: m x k, row-major, ldy >= k.  Element type FP64 for
 *   F64 values, FP32 for F32 and BF16 values, as for msrep_spmv.  Columns
 *   k..ld-1 are neither read nor written.  beta == 0: Y is not read.  X
 *   and Y must not overlap.  Each of X (n x ldx) and Y (m x ldy) must stay
 *   below 4 GiB (32-bit buffer offsets; MSREP_ERR_UNSUPPORTED otherwise).
 *   ws_d: msrep_spmm_ws_bytes(A, np, k) bytes of device memory (the FP64
 *   partial sums of split rows, 16 bytes per partition and column of a
 *   pass), caller-owned; its contents need not be kept between calls.
 *   All buffers are caller-owned device memory; kernels are launched on
 *   stream and nothing is synchronised.  k == 0 or m == 0 is a no-op.
 * Errors: MSREP_ERR_ARG (NULL pointers, np <= 0, k < 0, ld < k),
 * MSREP_ERR_SIZE (workspace too small), MSREP_ERR_UNSUPPORTED (format, X or
 * Y of 4 GiB or more).
 * Column j of Y equals msrep_spmv with x = column j of X up to the order of
 * the additions inside a partition.  k == 1 with ldx == ldy == 1 runs the
 * single-vector CSR kernel of msrep_spmv (default launch shape).
 */
size_t msrep_spmm_ws_bytes(const msrep_mat *A, int32_t np, int32_t k);
msrep_status msrep_spmm(const msrep_mat *A, const msrep_part *parts_d, const int32_t *lptr_d,
                        int32_t np, int32_t k, const void *X_d, int64_t ldx, void *Y_d,
                        int64_t ldy, double alpha, double beta, void *ws_d, size_t ws_bytes,
                        void *stream);

/* ------------------------------------------------------------- batched */
/*
 * A plan runs y_k = alpha*A_k*x_k + beta*y_k for count matrices in one
 * persistent launch captured in a hipGraph.  Each matrix is split into its
 * own equal-nnz partitions (np_k = ceil(nnz_k / tune_k.nnz_per_wave)); all
 * partitions go into one work list that resident wavefronts drain, followed
 * by one boundary-merge launch.  The plan keeps the partitions, the work list
 * and the descriptors in ws_d (caller memory, msrep_plan_ws_bytes bytes),
 * which must stay allocated until msrep_plan_destroy.  All matrices must
 * share one value type.  tunes may be NULL (defaults per matrix); the launch
 * shape (k_per_lane, waves_per_wg, and pipeline: 2 loads two chunks ahead,
 * otherwise one) comes from tunes[0], the partition size from each tune.
 * The merge of split rows is one segmented sum over the partitions of all
 * matrices (as in msrep_spmv).
 */
typedef struct msrep_plan_s *msrep_plan;

size_t msrep_plan_ws_bytes(int32_t count, const msrep_mat *mats,
                           const msrep_tune *tunes);
msrep_status msrep_plan_create(int32_t count, const msrep_mat *mats,
                               const msrep_tune *tunes, double alpha,
                               double beta, void *ws_d, size_t ws_bytes,
                               void *stream, msrep_plan *out);
/* x_ptrs / y_ptrs: host arrays of count device pointers (x_k: n_k values, y_k:
 * m_k values).  Stream-ordered; the pointer arrays are copied before return.
 * A plan holds one pointer table and one set of boundary carries, so calls
 * on one plan run one after another on the device even when issued on
 * different streams (each call's work waits for the previous call's). */
msrep_status msrep_spmv_batched(msrep_plan plan, const void *const *x_ptrs,
                                void *const *y_ptrs, void *stream);
/* Work items in the plan (partitions over all matrices). */
int64_t msrep_plan_items(msrep_plan plan);
msrep_status msrep_plan_destroy(msrep_plan plan);

/* --------------------------------------------------------------- serving */
/*
 * Continuous-batching server for the iterative-solver pattern: a request is
 * a matrix of a host pool plus `steps` SpMVs y_j = A*x_j against fresh x_j.
 * Matrices are uploaded into the caller's arena when the request is admitted
 * (admission is by bytes: matrix + partitions + vectors must fit in what the
 * arena has free) and stay resident while the request runs; a resident
 * matrix's partitions are built once, with its upload, and shared by every
 * request on it.  Every tick
 * executes the next steps of every active request (240 requests per tick at
 * most) in one batched launch, so requests that arrive while others run
 * join the next tick.  A request's steps are independent SpMVs: those that
 * share a tick are the columns of a multi-vector product Y = A*X, run as
 * passes of up to 8 columns side by side, so the matrix is read once per 8
 * steps rather than once per step.  A request reserves c = min(steps,
 * steps_per_tick) columns of X and Y (in blocks of 8, each block row-major;
 * 8 columns when c would take more than a sixteenth of the budget).
 * How many of them a tick runs follows the load: all that are left while
 * the tick is small against the GPU, else 8 per request.  Every tick but a
 * request's last runs a multiple of 8 of its steps, so its passes, and its
 * results, are bit-identical alone and in any mix, at any load and for
 * every steps_per_tick of 8 or more.  A request's descriptor is written to
 * the device once, when it is admitted; a tick only launches kernels.  Pool matrices are CSR of one value type with nnz < 2^31,
 * n < 2^24 and m < 2^26 (else MSREP_ERR_ARG).
 *   x_j[c] = 2*u - 1 with u the top 53 bits of splitmix64(key) / 2^53,
 *   key = seed ^ (rid << 40) ^ ((uint64)j << 24) ^ c (rid < 2^24, j < 2^16)
 *   (SplitMix64: Steele, Lea and Flood 2014), rounded to FP32 for F32 pools.
 * Latency of a request = its arrival (trace time) to the completion on the
 * device of its last step.  msrep_serve synchronises and returns when the
 * whole trace has drained.
 */
typedef struct msrep_host_mat {
  msrep_mat A;   /* CSR; ptr/idx/val are HOST pointers (pinned preferred)     */
  int32_t np;    /* partitions for this matrix (0: nnz_per_wave of the cfg)   */
  int32_t _pad;
} msrep_host_mat;

typedef struct msrep_serve_cfg {
  void *arena_d;        /* device memory the server allocates from           */
  size_t budget_bytes;  /* bytes of arena_d it may use                        */
  int32_t max_slots;    /* most requests active at once (1..4096)            */
  int32_t nnz_per_wave; /* partition size when a pool matrix has np == 0     */
  uint64_t seed;        /* x generator seed                                   */
  double time_scale;    /* trace seconds per wall second (1 = real time)     */
  int32_t keep_y;       /* msrep_serve: 1 copies every request's last y into  */
                        /* results[i].y_host (where not NULL)                */
  int32_t max_queue;    /* msrep_server_submit: most requests waiting for    */
                        /* admission before MSREP_ERR_BUSY (0: 2^20)          */
  int32_t steps_per_tick; /* most steps of one request in a tick (1..64;   */
                          /* 0: 64)                                          */
  int32_t _pad;
} msrep_serve_cfg;

typedef struct msrep_request {
  int64_t rid;        /* < 2^24                                              */
  double t_arrive;    /* seconds from the start of the trace                 */
  int32_t matrix;     /* index into the pool                                 */
  int32_t steps;      /* SpMVs, 1 .. 65535                                   */
} msrep_request;

typedef struct msrep_result {
  double t_arrive, t_admit, t_done; /* seconds on the trace clock            */
  int32_t status;                   /* MSREP_OK or an error                  */
  int32_t _pad;
  void *y_host;      /* keep_y: caller-provided host buffer of m values (set */
                     /* by the caller before the call, may be NULL)           */
} msrep_result;

typedef struct msrep_serve_stats {
  double p50_ms, p99_ms, mean_ms, max_ms; /* latency                          */
  double req_per_s, spmv_per_s;           /* over the makespan                */
  double makespan_s;
  double gflops;                          /* 2*nnz per SpMV over the makespan */
  int64_t n_done, n_failed, ticks;
  int64_t peak_bytes;                     /* most arena bytes in use          */
  int32_t peak_active;                    /* most requests active at once     */
  int32_t _pad;
} msrep_serve_stats;

msrep_status msrep_serve(const msrep_serve_cfg *cfg,
                         const msrep_host_mat *pool, int32_t pool_size,
                         const msrep_request *trace, int64_t n_req,
                         msrep_result *results, msrep_serve_stats *stats);

/* The same scheduler (admission, residency, eviction, continuous batching)
 * driven by a simulated device on a virtual clock instead of the GPU: an
 * upload takes bytes / upload_bytes_per_s, a tick takes tick_seconds plus
 * 2*nnz / flops_per_s for each step in it (values <= 0 keep defaults of
 * 25 GB/s, 500 GFLOP/s, 20 us).  No HIP call is made; cfg->arena_d may be
 * NULL and keep_y is ignored.  Results carry virtual times.  For testing the
 * scheduling logic without a GPU. */
msrep_status msrep_serve_simulate(const msrep_serve_cfg *cfg,
                                  const msrep_host_mat *pool, int32_t pool_size,
                                  const msrep_request *trace, int64_t n_req,
                                  msrep_result *results,
                                  msrep_serve_stats *stats,
                                  double upload_bytes_per_s, double flops_per_s,
                                  double tick_seconds);

/*
 * The same server taking requests as they come.  msrep_server_create copies
 * the configuration and the pool descriptors (the pool's host arrays and the
 * arena must stay valid until msrep_server_destroy) and starts the
 * scheduler on a thread of its own, bound to the device current at the call.
 *   msrep_server_submit: a request arrives now (req->t_arrive is ignored;
 *     arrival, admission and completion times are seconds on the server's
 *     clock, which starts at create).  y_host: NULL, or a host buffer of m
 *     values that receives the last y before the request is reported done.
 *     MSREP_ERR_BUSY when max_queue requests already wait; MSREP_ERR_ARG for
 *     a malformed request; the error that stopped the server otherwise.
 *   msrep_server_register: adds *mat (CSR of the pool's value type, host
 *     arrays the caller keeps valid until destroy, as for the pool) to the
 *     running server's pool and returns its index in *index, which requests
 *     may name from then on; the same checks as the pool at create
 *     (MSREP_ERR_ARG), the error that stopped the server otherwise.
 *   msrep_server_poll: up to cap completions (in completion order), waiting
 *     up to timeout_ms for the first when none is ready; returns how many
 *     were written, or a negative status when the server stopped on an
 *     error.  A request that can never fit the budget completes with status
 *     MSREP_ERR_BUDGET.
 *   msrep_server_destroy: waits until every submitted request has finished,
 *     stops the thread, frees the server and fills stats (may be NULL) over
 *     every completion; returns the error that stopped the server, if any.
 * Register, submit and poll may be called from any threads; destroy exactly
 * once.
 */
typedef struct msrep_server_s *msrep_server;

typedef struct msrep_completion {
  int64_t rid;                      /* the request's rid                    */
  double t_arrive, t_admit, t_done; /* seconds on the server's clock        */
  int32_t status;                   /* MSREP_OK or MSREP_ERR_BUDGET         */
  int32_t _pad;
} msrep_completion;

msrep_status msrep_server_create(const msrep_serve_cfg *cfg,
                                 const msrep_host_mat *pool, int32_t pool_size,
                                 msrep_server *out);
msrep_status msrep_server_submit(msrep_server server, const msrep_request *req,
                                 void *y_host);
msrep_status msrep_server_register(msrep_server server, const msrep_host_mat *mat,
                                   int32_t *index);
int64_t msrep_server_poll(msrep_server server, msrep_completion *out,
                          int64_t cap, int32_t timeout_ms);
msrep_status msrep_server_destroy(msrep_server server, msrep_serve_stats *stats);

/* Entry c of x_step for request rid (see msrep_serve), on the host. */
double msrep_serve_x_value(uint64_t seed, int64_t rid, int32_t step,
                           int64_t c);

/* The same x_step of request rid written on the device: x_d holds n values
 * (FP64 for MSREP_F64, FP32 for MSREP_F32, which rounds each value once),
 * launched on stream.  For callers that run a request's SpMVs themselves
 * (one msrep_spmv per step) with the server's inputs.  MSREP_ERR_ARG for a
 * NULL x_d with n > 0, n < 0 or another value type. */
msrep_status msrep_serve_fill_x(uint64_t seed, int64_t rid, int32_t step,
                                void *x_d, int32_t n, int32_t vtype,
                                void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MSREP_H */
