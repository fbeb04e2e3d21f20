"""Shared helpers of the GPU parity tests: put a synthetic matrix on the
device in a given format and value type, and compare results with the
oracle.  Format preparation for the inputs uses the (pinned) oracle
conversions; expected values come only from the oracle."""
from __future__ import annotations

import numpy as np

import oracle
import synth

F64_TOL = 1e-12   # |y - y_ref| <= F64_TOL * (|alpha||A||x| + |beta||y|)_i
F32_TOL = 1e-5


def host_formats(A):
    """(csr, csc, coo, coo_col) host arrays of a synth.Csr: CSR (ptr, col,
    val), CSC (ptr, row, val), row-sorted COO (row, col, val) and
    column-sorted COO (row, col, val in the CSC's order)."""
    cptr, crow, _, perm = oracle.transpose(A.m, A.n, A.ptr, A.col)
    rows = oracle.csr_to_coo(A.m, A.ptr)
    return {"csr": (A.ptr, A.col, A.val),
            "csc": (cptr, crow, A.val[perm]),
            "coo": (rows, A.col, A.val),
            "coo_col": (crow, oracle.csr_to_coo(A.n, cptr), A.val[perm])}


def stored_values(val64, vt):
    """Values as stored for value type vt, and their exact FP64 image."""
    import paper_2209_07552_amd as pk
    if vt == pk.F64:
        return val64, val64
    v32 = np.asarray(val64, np.float32)
    if vt == pk.F32:
        return v32, v32.astype(np.float64)
    bits = synth.bf16_bits(v32)
    return bits, synth.bf16_to_f64(bits)


def device_mat(A, fmt, vt):
    """Device Mat of A in format fmt ('csr'|'csc'|'coo'|'coo_col') and value type vt,
    plus the FP64 image of the stored values in that format's order."""
    import paper_2209_07552_amd as pk
    H = host_formats(A)
    a, b, v = H[fmt]
    sv, v64 = stored_values(v, vt)
    if fmt == "csr":
        M = pk.Mat(pk.CSR, vt, A.m, A.n, ptr=a, idx=b, val=sv)
    elif fmt == "csc":
        M = pk.Mat(pk.CSC, vt, A.m, A.n, ptr=a, idx=b, val=sv)
    elif fmt == "coo_col":
        M = pk.Mat(pk.COO_COL, vt, A.m, A.n, idx=a, idx2=b, val=sv)
    else:
        M = pk.Mat(pk.COO, vt, A.m, A.n, idx=a, idx2=b, val=sv)
    return M, v64


def oracle_y(A, fmt, v64, x64, alpha=1.0, beta=0.0, y_in=None):
    """Oracle result for the stored values (v64 in format order)."""
    H = host_formats(A)
    a, b, _ = H[fmt]
    if fmt == "csr":
        return oracle.spmv_csr(A.m, A.n, a, b, v64, x64, alpha, beta, y_in)
    if fmt == "csc":
        return oracle.spmv_csc(A.m, A.n, a, b, v64, x64, alpha, beta, y_in)
    return oracle.spmv_coo(A.m, A.n, a, b, v64, x64, alpha, beta, y_in)


def assert_close(y, ref, scale, tol, what=""):
    y = np.asarray(y, np.float64)
    err = np.abs(y - ref)
    bad = ~(err <= tol * scale)
    # rows whose scale is 0 must be exactly 0 (NaN-safe comparison above)
    if np.any(bad):
        i = int(np.argmax(bad))
        raise AssertionError("%s: %d rows out of tolerance; first row %d: got %r want %r "
                             "scale %r (tol %g)" % (what, int(bad.sum()), i, y[i], ref[i],
                                                    scale[i], tol))
    return float(np.max(err / np.where(scale > 0, scale, 1.0))) if len(y) else 0.0
