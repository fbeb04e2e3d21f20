"""Pins for the oracle's partition metadata (Sec. 3.2, Algorithms 2, 4, 6):
the hand-worked example, a linear-scan brute force on tiny matrices, the
invariants the paper states, and the partition-then-merge product."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from conftest import load_golden


def _golden_arrays():
    kv, parts = load_golden("example_6x6.txt")
    ints = ("row_ptr", "col_idx", "csc_col_ptr", "csc_row_idx", "coo_row_idx", "coocol_col_idx",
            "coocol_row_idx")
    g = {k: np.array(kv[k], dtype=np.int64) for k in ints}
    return int(kv["m"][0]), int(kv["n"][0]), g, parts


def _check_against(P, recs):
    for i, (fields, lp) in recs.items():
        got = [P.start_idx[i], P.end_idx[i], P.start_row[i], P.end_row[i], P.start_flag[i],
               P.end_flag[i], P.lptr_off[i]]
        assert [int(v) for v in got] == fields, (i, got, fields)
        if lp:
            assert list(P.local_ptr(i)) == lp, i


def test_golden_partitions(oracle_lib):
    m, n, g, parts = _golden_arrays()
    for (fmt, np_), recs in parts.items():
        split = "rows" if fmt.startswith("r") else "nnz"  # rcsr/rcsc/rcoo: the Baseline split
        if fmt[1:] == "csr":
            P = oracle.partition_ptr(m, g["row_ptr"], np_, split)
        elif fmt[1:] == "csc":
            P = oracle.partition_ptr(n, g["csc_col_ptr"], np_, split)
        elif fmt[1:] == "coocol":
            P = oracle.partition_coo_col(n, g["coocol_col_idx"], np_, split)
        else:
            P = oracle.partition_coo(m, g["coo_row_idx"], np_, split)
        assert len(recs) == np_
        _check_against(P, recs)
    P = oracle.partition_ptr(m, g["row_ptr"], 12)
    assert P.lptr_len == 29


def _brute(ptr, np_):
    """Linear-scan construction: every nonzero's row found by walking rows;
    local pointers counted element by element."""
    rows = len(ptr) - 1
    nnz = int(ptr[-1])
    row_of = []
    for r in range(rows):
        row_of += [r] * int(ptr[r + 1] - ptr[r])
    out = []
    # equal-nnz split: partition sizes q or q+1, the larger ones where the
    # running quota i*nnz/np crosses an integer (checked exactly below)
    bounds = [0]
    for i in range(1, np_ + 1):
        b = bounds[-1]
        while Fraction(b + 1) <= Fraction(i * nnz, np_):
            b += 1
        bounds.append(b)
    for i in range(np_):
        s, e = bounds[i], bounds[i + 1] - 1
        if s > e:
            sr = row_of[s] if s < nnz else rows
            out.append((s, e, sr, sr - 1, 0, 0, [0]))
            continue
        sr, er = row_of[s], row_of[e]
        sf = int(s > 0 and row_of[s - 1] == sr)
        ef = int(e + 1 < nnz and row_of[e + 1] == er)
        lp = [sum(1 for k in range(s, e + 1) if row_of[k] < sr + j) for j in range(er - sr + 2)]
        out.append((s, e, sr, er, sf, ef, lp))
    return out


def _tiny_ptrs(rng, count):
    yield np.zeros(1, np.int32)              # 0 x n
    yield np.zeros(4, np.int32)              # all rows empty
    yield np.array([0, 7], np.int32)         # one dense row
    yield np.array([0, 0, 0, 5, 5, 5], np.int32)
    for _ in range(count):
        rows = int(rng.integers(1, 9))
        cnt = rng.integers(0, 5, rows) * (rng.random(rows) < 0.7)
        yield np.concatenate([[0], np.cumsum(cnt)]).astype(np.int32)


def test_brute_force_tiny(oracle_lib):
    rng = np.random.default_rng(0)
    for ptr in _tiny_ptrs(rng, 60):
        nnz = int(ptr[-1])
        for np_ in range(1, nnz + 3):
            P = oracle.partition_ptr(len(ptr) - 1, ptr, np_)
            for i, (s, e, sr, er, sf, ef, lp) in enumerate(_brute(ptr, np_)):
                assert (P.start_idx[i], P.end_idx[i], P.start_row[i], P.end_row[i],
                        P.start_flag[i], P.end_flag[i]) == (s, e, sr, er, sf, ef), (ptr, np_, i)
                assert list(P.local_ptr(i)) == lp, (ptr, np_, i)


def _invariants(ptr, P):
    rows = len(ptr) - 1
    nnz = int(ptr[-1])
    np_ = P.np
    sizes = P.end_idx - P.start_idx + 1
    assert P.start_idx[0] == 0 and P.end_idx[-1] == nnz - 1
    assert np.all(P.start_idx[1:] == P.end_idx[:-1] + 1)      # contiguous, disjoint
    assert sizes.sum() == nnz
    assert set(np.unique(sizes)) <= {nnz // np_, -(-nnz // np_)}  # equal-nnz
    assert int((sizes == nnz // np_ + 1).sum()) == (nnz % np_ if nnz % np_ else 0)
    # offsets: non-overlapping, within rows + 2*np
    last_end = -1
    pieces = np.zeros(rows, np.int64)
    prev_nonempty = None
    for i in range(np_):
        lp = P.local_ptr(i)
        o = int(P.lptr_off[i])
        assert o > last_end
        last_end = o + len(lp) - 1
        assert last_end < oracle.lptr_bound(rows, np_)
        if sizes[i] == 0:
            assert list(lp) == [0] and P.start_flag[i] == 0 and P.end_flag[i] == 0
            continue
        s, sr, er = int(P.start_idx[i]), int(P.start_row[i]), int(P.end_row[i])
        assert ptr[sr] <= s < ptr[sr + 1]
        assert ptr[er] <= P.end_idx[i] < ptr[er + 1]
        assert lp[0] == 0 and lp[-1] == sizes[i] and np.all(np.diff(lp) >= 0)
        assert P.start_flag[i] == int(s > ptr[sr])
        if prev_nonempty is not None:
            j = prev_nonempty
            # the partial start row is inferred from the previous partition
            assert P.start_flag[i] == int(P.end_row[j] == sr)
            assert P.end_flag[j] == P.start_flag[i]
        pieces[sr:er + 1] += np.diff(lp)
        prev_nonempty = i
    if prev_nonempty is not None:
        assert P.end_flag[prev_nonempty] == 0
    # every row reassembles to its full length (pCSR -> CSR with no loss)
    assert np.array_equal(pieces, np.diff(ptr))


@pytest.mark.parametrize("np_", [1, 2, 3, 7, 8, 64, 1000, 5000])
def test_invariants_rmat(oracle_lib, np_):
    A, _ = synth.rmat_csr(scale=10, edge_factor=4, seed=1)
    P = oracle.partition_ptr(A.m, A.ptr, np_)
    _invariants(A.ptr, P)


def test_invariants_uniform_np8(oracle_lib):
    A, _ = synth.uniform_csr(4096, 4096, 16, seed=0)
    P = oracle.partition_ptr(A.m, A.ptr, 8)
    _invariants(A.ptr, P)
    # 65536 nnz / 8 = 8192 = exactly 512 rows of 16: no partial rows
    assert np.all(P.start_flag == 0) and np.all(P.end_flag == 0)
    for np_ in (3, 7):
        P = oracle.partition_ptr(A.m, A.ptr, np_)
        _invariants(A.ptr, P)
        assert P.start_flag.sum() > 0


def test_pcoo_matches_pcsr(oracle_lib):
    A, _ = synth.rmat_csr(scale=9, edge_factor=8, seed=2)
    row_idx = np.repeat(np.arange(A.m), np.diff(A.ptr)).astype(np.int32)
    for np_ in (1, 5, 64, 333, A.nnz + 3):
        P = oracle.partition_ptr(A.m, A.ptr, np_)
        Q = oracle.partition_coo(A.m, row_idx, np_)
        for f in ("start_idx", "end_idx", "start_row", "end_row", "start_flag", "end_flag"):
            assert np.array_equal(getattr(P, f), getattr(Q, f)), f


def test_pcsc_is_pcsr_of_transpose(oracle_lib):
    A, _ = synth.rmat_csr(scale=9, edge_factor=8, seed=3)
    S = sp.csr_matrix((A.val, A.col, A.ptr), shape=(A.m, A.n))
    C = S.tocsc()
    C.sort_indices()
    T = S.T.tocsr()
    T.sort_indices()
    for np_ in (4, 77):
        P = oracle.partition_ptr(A.n, C.indptr, np_)
        Q = oracle.partition_ptr(A.n, T.indptr, np_)
        for f in Partition_fields():
            assert np.array_equal(getattr(P, f), getattr(Q, f))
        assert np.array_equal(P.lptr[:P.lptr_len], Q.lptr[:Q.lptr_len])


def Partition_fields():
    return oracle.Partition.FIELDS


def test_rejects_unsorted_coo(oracle_lib):
    with pytest.raises(ValueError):
        oracle.partition_coo(3, np.array([0, 2, 1], np.int32), 2)
    with pytest.raises(ValueError):
        oracle.partition_ptr(3, np.array([0, 1, 2, 3], np.int32), 0)


def _partitioned_product(A, x, P, alpha, beta, y_in):
    """The method's product (Algorithm 3 with readings R8, R10): each
    partition computes its rows from its local pointer; split rows are merged
    by summing the partial sums in partition order; uncovered rows get
    beta*y.  Exact rational arithmetic, so any reading error shows."""
    m = A.m
    partial = {}
    for i in range(P.np):
        if P.end_idx[i] < P.start_idx[i]:
            continue
        s, sr = int(P.start_idx[i]), int(P.start_row[i])
        lp = P.local_ptr(i)
        for j in range(len(lp) - 1):
            acc = Fraction(0)
            for k in range(s + lp[j], s + lp[j + 1]):
                acc += Fraction(A.val[k]) * Fraction(x[A.col[k]])
            partial.setdefault(sr + j, []).append(acc)
    out = []
    for r in range(m):
        base = Fraction(beta) * Fraction(y_in[r]) if beta != 0 else Fraction(0)
        out.append(Fraction(alpha) * sum(partial.get(r, []), Fraction(0)) + base)
    return out


@pytest.mark.parametrize("np_", [1, 3, 8, 29, 200])
def test_partitioned_product_equals_spmv(oracle_lib, np_):
    rng = np.random.default_rng(np_)
    A, x = synth.rmat_csr(scale=6, edge_factor=3, seed=np_)
    y_in = rng.uniform(-1, 1, A.m)
    P = oracle.partition_ptr(A.m, A.ptr, np_)
    ex = _partitioned_product(A, x, P, 1.5, -0.5, y_in)
    y, s = oracle.spmv_csr(A.m, A.n, A.ptr, A.col, A.val, x, 1.5, -0.5, y_in)
    for r in range(A.m):
        assert abs(Fraction(y[r]) - ex[r]) <= Fraction(2.3e-16) * abs(ex[r]) + Fraction(1e-30)


def _rows_brute(ptr, np_):
    """The Baseline split by a scan: every nonzero's row found by walking the
    rows, each partition's nonzeros collected from the rows of its block."""
    rows = len(ptr) - 1
    row_of = []
    for r in range(rows):
        row_of += [r] * int(ptr[r + 1] - ptr[r])
    out = []
    for i in range(np_):
        block = set(range(i * rows // np_, (i + 1) * rows // np_))
        ks = [k for k, r in enumerate(row_of) if r in block]
        out.append(ks)
    return row_of, out


@pytest.mark.parametrize("seed", range(6))
def test_rows_split_brute_force(oracle_lib, seed):
    """Equal-rows (Baseline) records against a scan on tiny matrices with
    empty leading, trailing and interior rows, for every np from 1 to rows+2:
    each partition holds exactly the nonzeros of its row block, no flags, and
    its local pointer reassembles those rows."""
    rng = np.random.default_rng(seed)
    rows = int(rng.integers(1, 12))
    deg = rng.integers(0, 4, rows) * (rng.random(rows) < 0.7)
    ptr = np.concatenate([[0], np.cumsum(deg)]).astype(np.int32)
    for np_ in range(1, rows + 3):
        row_of, parts = _rows_brute(ptr, np_)
        P = oracle.partition_ptr(rows, ptr, np_, "rows")
        coo = np.array(row_of, np.int32)
        Q = oracle.partition_coo(rows, coo, np_, "rows")
        for i, ks in enumerate(parts):
            assert P.start_flag[i] == 0 and P.end_flag[i] == 0
            if ks:
                assert (P.start_idx[i], P.end_idx[i]) == (ks[0], ks[-1])
                assert ks == list(range(ks[0], ks[-1] + 1))
                assert (P.start_row[i], P.end_row[i]) == (row_of[ks[0]], row_of[ks[-1]])
                lp = P.local_ptr(i)
                for j, r in enumerate(range(P.start_row[i], P.end_row[i] + 1)):
                    assert lp[j + 1] - lp[j] == ptr[r + 1] - ptr[r]
            else:
                assert P.end_idx[i] == P.start_idx[i] - 1
                assert P.end_row[i] == P.start_row[i] - 1
                assert list(P.local_ptr(i)) == [0]
            for f in ("start_idx", "end_idx", "start_row", "end_row", "start_flag", "end_flag"):
                assert getattr(Q, f)[i] == getattr(P, f)[i], (f, i)


def test_rows_split_equals_nnz_split_when_rows_are_equal(oracle_lib):
    """With the same number of nonzeros in every row and np dividing the row
    count, equal row blocks are equal-nnz partitions: both splits agree."""
    A, _ = synth.uniform_csr(96, 80, 5, seed=4)
    for np_ in (1, 2, 3, 8, 12, 32, 96):
        P = oracle.partition_ptr(A.m, A.ptr, np_, "rows")
        Q = oracle.partition_ptr(A.m, A.ptr, np_)
        for f in Partition_FIELDS:
            assert np.array_equal(getattr(P, f), getattr(Q, f)), (np_, f)
        assert np.array_equal(P.lptr[:P.lptr_len], Q.lptr[:Q.lptr_len])


Partition_FIELDS = ("start_idx", "end_idx", "start_row", "end_row", "start_flag", "end_flag",
                    "lptr_off")


def test_golden_column_sorted_coo_arrays_and_product(oracle_lib):
    """The column-sorted COO of the hand-worked example is the CSC expanded
    (columns repeated by col_ptr), and the COO product over it gives the
    hand-worked y exactly."""
    kv, _ = load_golden("example_6x6.txt")
    m, n, g, _ = _golden_arrays()
    assert np.array_equal(oracle.csr_to_coo(n, g["csc_col_ptr"]), g["coocol_col_idx"])
    assert np.array_equal(g["coocol_row_idx"], g["csc_row_idx"])
    val = np.array(kv["csc_val"], np.float64)
    x = np.array(kv["x"], np.float64)
    y, _ = oracle.spmv_coo(m, n, g["coocol_row_idx"], g["coocol_col_idx"], val, x)
    assert np.array_equal(y, np.array(kv["y_a1_b0"], np.float64))


def test_column_sorted_coo_brute_force_tiny(oracle_lib):
    """pCOO on column-sorted COO against the linear-scan brute force, reading
    each tiny pointer as a column pointer: every np from 1 to nnz+2."""
    rng = np.random.default_rng(11)
    for cptr in _tiny_ptrs(rng, 60):
        cols = len(cptr) - 1
        nnz = int(cptr[-1])
        col_of = np.repeat(np.arange(cols), np.diff(cptr)).astype(np.int32)
        for np_ in range(1, nnz + 3):
            P = oracle.partition_coo_col(cols, col_of, np_)
            for i, (s, e, sc, ec, sf, ef, _) in enumerate(_brute(cptr, np_)):
                assert (P.start_idx[i], P.end_idx[i], P.start_row[i], P.end_row[i],
                        P.start_flag[i], P.end_flag[i], P.lptr_off[i]) == \
                    (s, e, sc, ec, sf, ef, 0), (cptr, np_, i)


def test_column_sorted_coo_matches_pcsc(oracle_lib):
    """The column-sorted split equals pCSC's records (Algorithm 4) of the
    same matrix, flags included, and its Baseline equals pCSC's Baseline."""
    A, _ = synth.rmat_csr(scale=9, edge_factor=8, seed=4)
    cptr, _, _, _ = oracle.transpose(A.m, A.n, A.ptr, A.col)
    col_of = oracle.csr_to_coo(A.n, cptr)
    for split in ("nnz", "rows"):
        for np_ in (1, 5, 64, 333, A.nnz + 3):
            P = oracle.partition_ptr(A.n, cptr, np_, split)
            Q = oracle.partition_coo_col(A.n, col_of, np_, split)
            for f in ("start_idx", "end_idx", "start_row", "end_row", "start_flag", "end_flag"):
                assert np.array_equal(getattr(P, f), getattr(Q, f)), (split, np_, f)


def test_rejects_column_unsorted_coo(oracle_lib):
    with pytest.raises(ValueError):
        oracle.partition_coo_col(3, np.array([0, 2, 1], np.int32), 2)
