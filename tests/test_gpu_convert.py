"""GPU parity of msrep_convert: every direction between CSR, CSC,
row-sorted COO and column-sorted COO, bit-exact against the oracle's stable conversions (indices
and values), on adversarial small matrices, at full R-MAT scale and on the
full-size stencil."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import host_formats, stored_values

torch = pytest.importorskip("torch")
pk = pytest.importorskip("paper_2209_07552_amd")

pytestmark = pytest.mark.gpu

FMT = {"csr": 0, "csc": 1, "coo": 2, "coo_col": 4}
COO_LIKE = ("coo", "coo_col")  # idx and idx2, no pointer


def _mk(A, fmt, vt):
    H = host_formats(A)
    a, b, v = H[fmt]
    sv, _ = stored_values(v, vt)
    if fmt in COO_LIKE:
        return pk.Mat(FMT[fmt], vt, A.m, A.n, idx=a, idx2=b, val=sv), H
    return pk.Mat(FMT[fmt], vt, A.m, A.n, ptr=a, idx=b, val=sv), H


def _host(M):
    torch.cuda.synchronize()
    f = lambda t: None if t is None else t.cpu().numpy()
    return f(M.ptr), f(M.idx), f(M.idx2), f(M.val)


def _check(A, src, dst, vt):
    M, H = _mk(A, src, vt)
    B = pk.msrep_convert(M, FMT[dst])
    ptr, idx, idx2, val = _host(B)
    a, b, v = H[dst]
    want_v, _ = stored_values(v, vt)
    want_v = np.asarray(want_v)
    if dst in COO_LIKE:
        assert np.array_equal(idx, a) and np.array_equal(idx2, b), (A.name, src, dst)
    else:
        assert np.array_equal(ptr, a) and np.array_equal(idx, b), (A.name, src, dst)
    got_v = val.view(np.uint16) if vt == pk.BF16 else val
    assert np.array_equal(got_v, want_v), (A.name, src, dst, vt)


def _small_set():
    rng = np.random.default_rng(9)
    out = []
    for counts, n in (([0, 0, 0], 4), ([5], 7), ([0, 3, 0, 0, 2, 0], 5), ([], 3)):
        counts = np.asarray(counts, np.int64)
        cols = np.concatenate([np.sort(rng.choice(n, c, replace=False)) for c in counts]) \
            if counts.sum() else np.zeros(0, np.int64)
        ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
        out.append(synth.Csr(len(counts), n, ptr, cols.astype(np.int32),
                             rng.uniform(-1, 1, len(cols)), name="small%d" % len(out)))
    out.append(synth.uniform_csr(300, 1000, 7, seed=3)[0])
    out.append(synth.uniform_csr(1000, 200, 9, seed=4)[0])
    return out


@pytest.mark.parametrize("src", ["csr", "csc", "coo", "coo_col"])
@pytest.mark.parametrize("dst", ["csr", "csc", "coo", "coo_col"])
def test_convert_small(src, dst):
    for A in _small_set():
        for vt in (0, 1, 2):
            _check(A, src, dst, vt)


@pytest.mark.parametrize("src,dst", [("csr", "csc"), ("csc", "csr"), ("csr", "coo"),
                                     ("coo", "csr"), ("coo", "csc"), ("csc", "coo"),
                                     ("csr", "coo_col"), ("coo_col", "csr"), ("csc", "coo_col"),
                                     ("coo_col", "csc"), ("coo", "coo_col"), ("coo_col", "coo")])
def test_convert_rmat(src, dst):
    A, _ = synth.rmat_csr(scale=16, edge_factor=16, seed=7)
    _check(A, src, dst, pk.F64)


def test_round_trip_rmat20():
    A, _ = synth.rmat_csr(scale=20, edge_factor=16, seed=0)
    M, H = _mk(A, "csr", pk.F64)
    C = pk.msrep_convert(M, pk.CSC)
    O = pk.msrep_convert(C, pk.COO)
    R = pk.msrep_convert(O, pk.CSR)
    ptr, idx, _, val = _host(R)
    assert np.array_equal(ptr, A.ptr) and np.array_equal(idx, A.col) and np.array_equal(val, A.val)
    cptr, cidx, _, cval = _host(C)
    a, b, v = H["csc"]
    assert np.array_equal(cptr, a) and np.array_equal(cidx, b) and np.array_equal(cval, v)


def test_duplicates_keep_storage_order():
    # duplicate (row, col) entries: the transpose is stable
    ptr = np.array([0, 3, 4], np.int32)
    col = np.array([1, 1, 0, 1], np.int32)
    val = np.array([10.0, 20.0, 30.0, 40.0])
    M = pk.Mat(pk.CSR, pk.F64, 2, 2, ptr=ptr, idx=col, val=val)
    p, i, _, v = _host(pk.msrep_convert(M, pk.CSC))
    cptr, crow, cval, _ = oracle.transpose(2, 2, ptr, col, val)
    assert np.array_equal(p, cptr) and np.array_equal(i, crow) and np.array_equal(v, cval)


def test_round_trip_column_sorted_rmat20():
    """CSR -> column-sorted COO -> CSC -> row-sorted COO -> CSR returns the
    input bit for bit at R-MAT scale 20; the column-sorted arrays equal the
    oracle's (the CSC expanded)."""
    A, _ = synth.rmat_csr(scale=20, edge_factor=16, seed=0)
    M, H = _mk(A, "csr", pk.F64)
    K = pk.msrep_convert(M, pk.COO_COL)
    _, kr, kc, kv = _host(K)
    a, b, v = H["coo_col"]
    assert np.array_equal(kr, a) and np.array_equal(kc, b) and np.array_equal(kv, v)
    R = pk.msrep_convert(pk.msrep_convert(pk.msrep_convert(K, pk.CSC), pk.COO), pk.CSR)
    ptr, idx, _, val = _host(R)
    assert np.array_equal(ptr, A.ptr) and np.array_equal(idx, A.col) and np.array_equal(val, A.val)


def test_convert_stencil_full_size():
    """The benchmark's 256^3 stencil (117M nonzeros, 2^24 rows): CSR -> CSC and
    CSR -> row-sorted COO bit-exact against the oracle's conversions (the
    stencil is symmetric, so its CSC arrays also equal its CSR arrays)."""
    A, _ = synth.stencil7_csr(256, seed=0)
    M = pk.Mat(pk.CSR, pk.F64, A.m, A.n, ptr=A.ptr, idx=A.col, val=A.val)
    C = pk.msrep_convert(M, pk.CSC)
    cptr, crow, _, cval = _host(C)
    del C
    optr, orow, _, perm = oracle.transpose(A.m, A.n, A.ptr, A.col)
    assert np.array_equal(cptr, optr) and np.array_equal(crow, orow)
    assert np.array_equal(cval, A.val[perm])
    assert np.array_equal(cptr, A.ptr) and np.array_equal(crow, A.col)
    del cptr, crow, cval, optr, orow, perm
    O = pk.msrep_convert(M, pk.COO)
    _, r, c, v = _host(O)
    assert np.array_equal(r, oracle.csr_to_coo(A.m, A.ptr))
    assert np.array_equal(c, A.col) and np.array_equal(v, A.val)
    del O, M
    torch.cuda.empty_cache()


def _any_order(A, rng):
    """A's entries as COO in a seeded random order: (rows, cols, vals)."""
    rows = oracle.csr_to_coo(A.m, A.ptr)
    sh = rng.permutation(A.nnz)
    return rows[sh], A.col[sh], A.val[sh]


def _expect_from_any(m, n, r, c, v, dst):
    """The oracle's sorted arrays for COO in any order converted to dst."""
    if dst in ("csr", "coo"):
        p = oracle.coo_sort(m, n, r, c)
        if dst == "coo":
            return r[p], c[p], v[p]
        return oracle.coo_to_csr(m, r[p]), c[p], v[p]
    p = oracle.coo_sort(n, m, c, r)
    if dst == "coo_col":
        return r[p], c[p], v[p]
    return oracle.coo_to_csr(n, c[p]), r[p], v[p]


@pytest.mark.parametrize("dst", ["csr", "csc", "coo", "coo_col"])
@pytest.mark.parametrize("vt", [0, 1, 2])
def test_convert_from_any_order(dst, vt):
    """COO in any order into every sorted format, bit-exact against the
    oracle's sort (ties by the other index, then storage order), on the small
    adversarial set, duplicates, and R-MAT 16 shuffled."""
    rng = np.random.default_rng(5)
    mats = _small_set() + [synth.rmat_csr(scale=16, edge_factor=16, seed=7)[0]]
    for A in mats:
        r, c, v = _any_order(A, rng)
        if A.nnz > 4:  # duplicates: repeat a few entries with other values
            k = rng.integers(0, A.nnz, 4)
            r, c = np.concatenate([r, r[k]]), np.concatenate([c, c[k]])
            v = np.concatenate([v, rng.uniform(-1, 1, 4)])
        sv, _ = stored_values(v, vt)
        M = pk.Mat(pk.COO_ANY, vt, A.m, A.n, idx=r, idx2=c, val=sv)
        B = pk.msrep_convert(M, FMT[dst])
        ptr, idx, idx2, val = _host(B)
        a, b, want = _expect_from_any(A.m, A.n, r, c, np.asarray(sv), dst)
        got_v = val.view(np.uint16) if vt == pk.BF16 else val
        if dst in COO_LIKE:
            assert np.array_equal(idx, a) and np.array_equal(idx2, b), (A.name, dst)
        else:
            assert np.array_equal(ptr, a) and np.array_equal(idx, b), (A.name, dst)
        assert np.array_equal(got_v, want), (A.name, dst, vt)


def test_convert_from_any_order_rmat20_round_trip():
    """R-MAT scale 20 shuffled and sorted back: CSR bit for bit."""
    A, _ = synth.rmat_csr(scale=20, edge_factor=16, seed=0)
    r, c, v = _any_order(A, np.random.default_rng(3))
    M = pk.Mat(pk.COO_ANY, pk.F64, A.m, A.n, idx=r, idx2=c, val=v)
    ptr, idx, _, val = _host(pk.msrep_convert(M, pk.CSR))
    assert np.array_equal(ptr, A.ptr) and np.array_equal(idx, A.col) and np.array_equal(val, A.val)


def _tridiagonal(m, seed):
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(m), 3) + np.tile([-1, 0, 1], m)
    cols = np.repeat(np.arange(m), 3)
    keep = (rows >= 0) & (rows < m)
    r, c = cols[keep], rows[keep]  # row-major: row i holds i-1, i, i+1
    ptr = np.concatenate([[0], np.cumsum(np.bincount(r, minlength=m))]).astype(np.int32)
    return synth.Csr(m, m, ptr, c.astype(np.int32), rng.uniform(-1, 1, len(c)),
                     name="tridiagonal%d" % m)


@pytest.mark.parametrize("src,dst", [("csr", "csc"), ("csc", "csr"), ("coo", "coo_col"),
                                     ("coo_col", "csr")])
@pytest.mark.parametrize("vt", [0, 1, 2])
def test_transpose_both_strategies(src, dst, vt):
    """A transposing conversion sorts (key, position) pairs and gathers the
    entries when the matrix is banded (9 in 10 sampled entries with row and
    column within max(m, n)/64), and moves whole entries through the sort
    otherwise: banded matrices (a 64^3 stencil, a tridiagonal one) take the
    first, uniform random ones the second; all bit-exact."""
    mats = [synth.stencil7_csr(g=64, seed=5)[0], _tridiagonal(5000, 6),
            synth.uniform_csr(5000, 5000, 9, seed=7)[0], synth.uniform_csr(64, 300, 5, seed=8)[0]]
    for A in mats:
        _check(A, src, dst, vt)
