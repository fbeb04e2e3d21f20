"""Pins for the oracle's format conversions (Sec. 2.1): scipy.sparse (a
library reduction with a unique canonical answer), round trips and the
hand-worked example."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from conftest import load_golden


def test_golden(oracle_lib):
    kv, _ = load_golden("example_6x6.txt")
    m, n = int(kv["m"][0]), int(kv["n"][0])
    ptr = np.array(kv["row_ptr"], np.int32)
    col = np.array(kv["col_idx"], np.int32)
    val = np.array(kv["val"], np.float64)
    cptr, crow, cval, perm = oracle.transpose(m, n, ptr, col, val)
    assert list(cptr) == [int(v) for v in kv["csc_col_ptr"]]
    assert list(crow) == [int(v) for v in kv["csc_row_idx"]]
    assert list(cval) == [float(v) for v in kv["csc_val"]]
    assert np.array_equal(val[perm], cval)
    assert list(oracle.csr_to_coo(m, ptr)) == [int(v) for v in kv["coo_row_idx"]]
    assert np.array_equal(oracle.coo_to_csr(m, oracle.csr_to_coo(m, ptr)), ptr)


@pytest.mark.parametrize("kind", ["uniform", "rmat", "rect"])
def test_vs_scipy_and_round_trips(oracle_lib, kind):
    if kind == "uniform":
        A, _ = synth.uniform_csr(700, 700, 9, seed=1)
    elif kind == "rmat":
        A, _ = synth.rmat_csr(scale=11, edge_factor=8, seed=1)
    else:
        A, _ = synth.uniform_csr(300, 1200, 5, seed=2)
    S = sp.csr_matrix((A.val, A.col, A.ptr), shape=(A.m, A.n))
    C = S.tocsc()
    C.sort_indices()
    cptr, crow, cval, perm = oracle.transpose(A.m, A.n, A.ptr, A.col, A.val)
    assert np.array_equal(cptr, C.indptr) and np.array_equal(crow, C.indices)
    assert np.array_equal(cval, C.data) and np.array_equal(A.val[perm], cval)
    # CSC -> CSR is the same stable transpose with the roles swapped
    rptr, rcol, rval, _ = oracle.transpose(A.n, A.m, cptr, crow, cval)
    assert np.array_equal(rptr, A.ptr) and np.array_equal(rcol, A.col)
    assert np.array_equal(rval, A.val)
    # CSR <-> COO
    O = S.tocoo()
    ri = oracle.csr_to_coo(A.m, A.ptr)
    assert np.array_equal(ri, O.row) and np.array_equal(A.col, O.col)
    assert np.array_equal(oracle.coo_to_csr(A.m, ri), A.ptr)
    # COO -> CSC -> COO
    crow2 = oracle.csr_to_coo(A.n, cptr)  # column index of every CSC entry
    OC = S.tocsc().tocoo()
    order = np.lexsort((OC.row, OC.col))
    assert np.array_equal(crow2, OC.col[order]) and np.array_equal(crow, OC.row[order])


def test_stable_with_duplicates(oracle_lib):
    """Duplicate (row, col) entries keep their storage order."""
    ptr = np.array([0, 3, 4], np.int32)
    col = np.array([1, 1, 0, 1], np.int32)
    val = np.array([10.0, 20.0, 30.0, 40.0])
    cptr, crow, cval, perm = oracle.transpose(2, 2, ptr, col, val)
    assert list(cptr) == [0, 1, 4]
    assert list(crow) == [0, 0, 0, 1]
    assert list(cval) == [30.0, 10.0, 20.0, 40.0]
    assert list(perm) == [2, 0, 1, 3]


def test_coo_to_csr_rejects_unsorted(oracle_lib):
    with pytest.raises(ValueError):
        oracle.coo_to_csr(3, np.array([1, 0], np.int32))


def test_coo_sort_hand_example(oracle_lib):
    """COO in any order sorted by (row, column): worked by hand, with a
    duplicate (row 1, column 2) whose two entries keep their storage order,
    and the same entries sorted by (column, row)."""
    row = np.array([2, 1, 0, 1, 2, 1], np.int32)
    col = np.array([0, 2, 1, 0, 2, 2], np.int32)
    # by (row, col): (0,1)@2, (1,0)@3, (1,2)@1, (1,2)@5, (2,0)@0, (2,2)@4
    assert list(oracle.coo_sort(3, 3, row, col)) == [2, 3, 1, 5, 0, 4]
    # by (col, row): (0,1)@3, (0,2)@0, (1,0)@2, (2,1)@1, (2,1)@5, (2,2)@4
    assert list(oracle.coo_sort(3, 3, col, row)) == [3, 0, 2, 1, 5, 4]
    assert len(oracle.coo_sort(4, 4, np.zeros(0, np.int32), np.zeros(0, np.int32))) == 0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_coo_sort_vs_numpy_lexsort(oracle_lib, seed):
    """Against numpy's stable lexicographic sort (a library routine with a
    unique answer for a stable order), on shuffled entries with many
    duplicates, in both key orders; the sorted triples equal the CSR /
    CSC the oracle's own conversions give for the deduplicated-free case."""
    rng = np.random.default_rng(seed)
    m, n, nnz = 57, 31, 2000
    row = rng.integers(0, m, nnz).astype(np.int32)
    col = rng.integers(0, n, nnz).astype(np.int32)
    p = oracle.coo_sort(m, n, row, col)
    assert np.array_equal(p, np.lexsort((col, row)))
    q = oracle.coo_sort(n, m, col, row)
    assert np.array_equal(q, np.lexsort((row, col)))
    # a CSR matrix shuffled and sorted back gives its CSR arrays
    A, _ = synth.uniform_csr(200, 150, 9, seed=seed)
    rows = oracle.csr_to_coo(A.m, A.ptr)
    sh = rng.permutation(A.nnz)
    back = oracle.coo_sort(A.m, A.n, rows[sh], A.col[sh])
    assert np.array_equal(rows[sh][back], rows) and np.array_equal(A.col[sh][back], A.col)
    cptr, crow, _, _ = oracle.transpose(A.m, A.n, A.ptr, A.col)
    bc = oracle.coo_sort(A.n, A.m, A.col[sh], rows[sh])
    assert np.array_equal(rows[sh][bc], crow)
    assert np.array_equal(oracle.coo_to_csr(A.n, A.col[sh][bc]), cptr)


def test_coo_sort_rejects_out_of_range(oracle_lib):
    with pytest.raises(ValueError):
        oracle.coo_sort(2, 2, np.array([0, 2], np.int32), np.array([0, 0], np.int32))
