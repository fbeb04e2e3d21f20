"""FP64 CPU oracle for the equal-nnz partitioned SpMV of msRep (arXiv 2209.07552).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports it,
and it imports nothing from the product library.

The arithmetic lives in ``msrep_oracle.c`` (plain C, FP64, Dot2 row sums);
this module compiles it with gcc and marshals numpy arrays through ctypes.
Every function cites, in the C source, the passage of the paper it follows.

Pins (tests/test_oracle_*.py check this oracle against values fixed by the
paper or by mathematics, never against itself):
  * SpMM (several right-hand sides): numpy dense products and exact
    rational arithmetic on small cases, and its columns against the SpMV
    pins' closed forms (stencil times ones).
  * SpMV: exact rational arithmetic (fractions) on small random matrices,
    numpy dense products, scipy.sparse, identity / permutation / diagonal
    special cases, the 7-point stencil times ones in closed form, dyadic
    inputs whose sums are exact, and a hand-worked example
    (tests/golden/example_6x6.txt).
  * Partition metadata: a linear-scan brute force on tiny matrices, the
    invariants the paper states (contiguous, disjoint, equal-nnz, start flag,
    reassembly of every row) and the hand-worked example.
  * Conversions: scipy.sparse tocsc/tocsr/tocoo, and round trips.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "msrep_oracle.c")
# ORACLE_LIB selects another build (the sanitizer build, build_sanitized()).
_LIB = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

OK = 0
ERR_ARG = -1
ERR_FORMAT = -2
ERR_SIZE = -3


def build(force: bool = True) -> str:
    """Compile the oracle into oracle/liboracle.so with gcc and return its path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = ctypes.CDLL(_LIB)
        i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        vp = ctypes.c_void_p
        _lib.oracle_spmv_csr.argtypes = [i32, i32, vp, vp, vp, vp, dbl, dbl, vp, vp, vp]
        _lib.oracle_spmv_csr_plain.argtypes = [i32, i32, vp, vp, vp, vp, dbl, dbl, vp, vp, i32]
        _lib.oracle_spmm_csr.argtypes = [i32, i32, i32, vp, vp, vp, vp, i64, dbl, dbl, vp, i64,
                                         vp, vp]
        _lib.oracle_spmv_csc.argtypes = [i32, i32, vp, vp, vp, vp, dbl, dbl, vp, vp, vp]
        _lib.oracle_spmv_coo.argtypes = [i32, i32, i64, vp, vp, vp, vp, dbl, dbl, vp, vp, vp]
        _lib.oracle_partition_ptr.argtypes = [i32, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, i64, vp]
        _lib.oracle_partition_coo.argtypes = [i32, i64, vp, i32, vp, vp, vp, vp, vp, vp, vp]
        _lib.oracle_partition_rows_ptr.argtypes = _lib.oracle_partition_ptr.argtypes
        _lib.oracle_partition_rows_coo.argtypes = _lib.oracle_partition_coo.argtypes
        _lib.oracle_partition_coo_col.argtypes = _lib.oracle_partition_coo.argtypes
        _lib.oracle_partition_cols_coo_col.argtypes = _lib.oracle_partition_coo.argtypes
        _lib.oracle_csr_to_coo.argtypes = [i32, vp, vp]
        _lib.oracle_coo_to_csr.argtypes = [i32, i64, vp, vp]
        _lib.oracle_transpose.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp]
        _lib.oracle_coo_sort.argtypes = [i32, i32, i64, vp, vp, vp]
        for f in ("oracle_spmv_csr", "oracle_spmv_csr_plain", "oracle_spmm_csr", "oracle_spmv_csc", "oracle_spmv_coo",
                  "oracle_partition_ptr", "oracle_partition_coo", "oracle_partition_rows_ptr",
                  "oracle_partition_rows_coo", "oracle_partition_coo_col",
                  "oracle_partition_cols_coo_col", "oracle_csr_to_coo",
                  "oracle_coo_to_csr", "oracle_transpose", "oracle_coo_sort"):
            getattr(_lib, f).restype = ctypes.c_int
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _check(rc, what):
    if rc != OK:
        raise ValueError("oracle %s failed with status %d" % (what, rc))


def _yin(y_in, m, beta):
    if beta == 0.0:
        return None
    return _c(y_in, np.float64)


def spmv_csr(m, n, row_ptr, col_idx, val, x, alpha=1.0, beta=0.0, y_in=None):
    """y = alpha*A*x + beta*y_in for CSR A; returns (y, scale) with
    scale_i = |alpha|*(|A||x|)_i + |beta|*|y_in_i|."""
    lib = _load()
    row_ptr, col_idx = _c(row_ptr, np.int32), _c(col_idx, np.int32)
    val, x = _c(val, np.float64), _c(x, np.float64)
    yi = _yin(y_in, m, beta)
    y = np.empty(m, np.float64)
    s = np.empty(m, np.float64)
    _check(lib.oracle_spmv_csr(m, n, _p(row_ptr), _p(col_idx), _p(val), _p(x), alpha, beta,
                               _p(yi), _p(y), _p(s)), "spmv_csr")
    return y, s


def spmv_csr_plain(m, n, row_ptr, col_idx, val, x, alpha=1.0, beta=0.0, y_in=None,
                   threads=1):
    """The uncompensated CSR row loop (plain FP64 sums) on `threads` OpenMP
    threads: the CPU baseline's arithmetic.  Returns y."""
    lib = _load()
    row_ptr, col_idx = _c(row_ptr, np.int32), _c(col_idx, np.int32)
    val, x = _c(val, np.float64), _c(x, np.float64)
    yi = _yin(y_in, m, beta)
    y = np.empty(m, np.float64)
    _check(lib.oracle_spmv_csr_plain(m, n, _p(row_ptr), _p(col_idx), _p(val), _p(x), alpha, beta,
                                     _p(yi), _p(y), int(threads)), "spmv_csr_plain")
    return y


def spmm_csr(m, n, row_ptr, col_idx, val, X, alpha=1.0, beta=0.0, Y_in=None):
    """Y = alpha*A*X + beta*Y_in for CSR A and the k columns of X (n x k);
    returns (Y, scale), both m x k, scale = |alpha|*(|A||X|) + |beta|*|Y_in|."""
    lib = _load()
    row_ptr, col_idx = _c(row_ptr, np.int32), _c(col_idx, np.int32)
    val = _c(val, np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    if X.ndim != 2 or X.shape[0] != n:
        raise ValueError("X must be n x k")
    k = X.shape[1]
    if beta != 0.0:
        Yi = np.ascontiguousarray(Y_in, dtype=np.float64)
        if Yi.shape != (m, k):
            raise ValueError("Y_in must be m x k")
    else:
        Yi = np.zeros((m, k), np.float64)
    Y = np.empty((m, k), np.float64)
    S = np.empty((m, k), np.float64)
    _check(lib.oracle_spmm_csr(m, n, k, _p(row_ptr), _p(col_idx), _p(val), _p(X), k, alpha,
                               beta, _p(Yi), k, _p(Y), _p(S)), "spmm_csr")
    return Y, S


def spmv_csc(m, n, col_ptr, row_idx, val, x, alpha=1.0, beta=0.0, y_in=None):
    lib = _load()
    col_ptr, row_idx = _c(col_ptr, np.int32), _c(row_idx, np.int32)
    val, x = _c(val, np.float64), _c(x, np.float64)
    yi = _yin(y_in, m, beta)
    y = np.empty(m, np.float64)
    s = np.empty(m, np.float64)
    _check(lib.oracle_spmv_csc(m, n, _p(col_ptr), _p(row_idx), _p(val), _p(x), alpha, beta,
                               _p(yi), _p(y), _p(s)), "spmv_csc")
    return y, s


def spmv_coo(m, n, row_idx, col_idx, val, x, alpha=1.0, beta=0.0, y_in=None):
    lib = _load()
    row_idx, col_idx = _c(row_idx, np.int32), _c(col_idx, np.int32)
    val, x = _c(val, np.float64), _c(x, np.float64)
    yi = _yin(y_in, m, beta)
    y = np.empty(m, np.float64)
    s = np.empty(m, np.float64)
    _check(lib.oracle_spmv_coo(m, n, len(row_idx), _p(row_idx), _p(col_idx), _p(val), _p(x),
                               alpha, beta, _p(yi), _p(y), _p(s)), "spmv_coo")
    return y, s


class Partition:
    """Partition metadata as numpy arrays (one entry per partition) plus the
    local pointer array ``lptr`` (partition i's entries start at lptr_off[i])."""

    FIELDS = ("start_idx", "end_idx", "start_row", "end_row", "start_flag", "end_flag",
              "lptr_off")

    def __init__(self, np_):
        self.np = np_
        self.start_idx = np.zeros(np_, np.int64)
        self.end_idx = np.zeros(np_, np.int64)
        self.start_row = np.zeros(np_, np.int32)
        self.end_row = np.zeros(np_, np.int32)
        self.start_flag = np.zeros(np_, np.int32)
        self.end_flag = np.zeros(np_, np.int32)
        self.lptr_off = np.zeros(np_, np.int64)
        self.lptr = np.zeros(0, np.int32)
        self.lptr_len = 0

    def local_ptr(self, i):
        """Partition i's local pointer (R_i + 1 entries)."""
        r = int(self.end_row[i]) - int(self.start_row[i]) + 1
        o = int(self.lptr_off[i])
        return self.lptr[o:o + r + 1]


def lptr_bound(rows, np_):
    """Entries the local-pointer array needs: rows + 2*np."""
    return int(rows) + 2 * int(np_)


def partition_ptr(rows, ptr, np_, split="nnz"):
    """pCSR (ptr = CSR row_ptr, Algorithm 2) or pCSC (ptr = CSC col_ptr,
    Algorithm 4); split="rows": the Baseline's equal row blocks (Sec. 5.3)."""
    lib = _load()
    fn = lib.oracle_partition_rows_ptr if split == "rows" else lib.oracle_partition_ptr
    ptr = _c(ptr, np.int32)
    P = Partition(np_)
    cap = lptr_bound(rows, np_)
    P.lptr = np.full(cap, -1, np.int32)
    ln = np.zeros(1, np.int64)
    _check(fn(rows, _p(ptr), np_, _p(P.start_idx), _p(P.end_idx),
                                    _p(P.start_row), _p(P.end_row), _p(P.start_flag),
                                    _p(P.end_flag), _p(P.lptr_off), _p(P.lptr), cap, _p(ln)),
           "partition_ptr")
    P.lptr_len = int(ln[0])
    return P


def partition_coo(rows, row_idx, np_, split="nnz"):
    """pCOO on row-sorted COO (Algorithm 6); split="rows": the Baseline's
    equal row blocks (Sec. 5.3)."""
    lib = _load()
    fn = lib.oracle_partition_rows_coo if split == "rows" else lib.oracle_partition_coo
    row_idx = _c(row_idx, np.int32)
    P = Partition(np_)
    _check(fn(rows, len(row_idx), _p(row_idx), np_, _p(P.start_idx),
                                    _p(P.end_idx), _p(P.start_row), _p(P.end_row),
                                    _p(P.start_flag), _p(P.end_flag), _p(P.lptr_off)),
           "partition_coo")
    return P


def partition_coo_col(cols, col_idx, np_, split="nnz"):
    """pCOO on column-sorted COO (Sec. 3.2.3, Algorithm 6 on the column
    index; start_row / end_row hold columns); split="rows": the Baseline's
    equal column blocks (Sec. 5.3)."""
    lib = _load()
    fn = (lib.oracle_partition_cols_coo_col if split == "rows"
          else lib.oracle_partition_coo_col)
    col_idx = _c(col_idx, np.int32)
    P = Partition(np_)
    _check(fn(cols, len(col_idx), _p(col_idx), np_, _p(P.start_idx), _p(P.end_idx),
              _p(P.start_row), _p(P.end_row), _p(P.start_flag), _p(P.end_flag),
              _p(P.lptr_off)), "partition_coo_col")
    return P


def csr_to_coo(m, row_ptr):
    """Row indices of every nonzero (columns and values keep their order)."""
    lib = _load()
    row_ptr = _c(row_ptr, np.int32)
    row_idx = np.empty(int(row_ptr[m]), np.int32)
    _check(lib.oracle_csr_to_coo(m, _p(row_ptr), _p(row_idx)), "csr_to_coo")
    return row_idx


def coo_to_csr(m, row_idx):
    lib = _load()
    row_idx = _c(row_idx, np.int32)
    row_ptr = np.empty(m + 1, np.int32)
    _check(lib.oracle_coo_to_csr(m, len(row_idx), _p(row_idx), _p(row_ptr)), "coo_to_csr")
    return row_ptr


def coo_sort(n_major, n_minor, major, minor):
    """The storage positions of COO entries given in any order, sorted by
    (major, minor); entries equal on both keep their storage order."""
    lib = _load()
    major, minor = _c(major, np.int32), _c(minor, np.int32)
    perm = np.empty(len(major), np.int64)
    _check(lib.oracle_coo_sort(int(n_major), int(n_minor), len(major), _p(major), _p(minor),
                               _p(perm)), "coo_sort")
    return perm


def transpose(m, n, row_ptr, col_idx, val=None):
    """Stable compressed transpose: CSR (m x n) -> CSC, or CSC -> CSR with the
    roles swapped.  Returns (col_ptr, row_idx, val_out or None, perm)."""
    lib = _load()
    row_ptr, col_idx = _c(row_ptr, np.int32), _c(col_idx, np.int32)
    nnz = int(row_ptr[m])
    col_ptr = np.empty(n + 1, np.int32)
    row_idx = np.empty(nnz, np.int32)
    perm = np.empty(nnz, np.int64)
    v = None if val is None else _c(val, np.float64)
    vo = None if val is None else np.empty(nnz, np.float64)
    _check(lib.oracle_transpose(m, n, _p(row_ptr), _p(col_idx), _p(v), _p(col_ptr),
                                _p(row_idx), _p(vo), _p(perm)), "transpose")
    return col_ptr, row_idx, vo, perm
