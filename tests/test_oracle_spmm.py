"""Pins for the oracle's product with several right-hand sides (Algorithm 1
applied to every column of a row-major block X): the hand-worked example,
exact rational sums, numpy dense products, the 7-point stencil times constant
columns in closed form, and leading dimensions wider than k.  None of these
compares the oracle with itself."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from conftest import load_golden

EPS = np.finfo(np.float64).eps


def _random_csr(rng, m, n, density):
    dense = rng.uniform(-1, 1, (m, n)) * (rng.random((m, n)) < density)
    if m > 2:
        dense[rng.integers(0, m, size=max(1, m // 4))] = 0.0
    A = sp.csr_matrix(dense)
    A.sort_indices()
    return A, dense


def test_golden_two_columns(oracle_lib):
    kv, _ = load_golden("example_6x6.txt")
    m, n = int(kv["m"][0]), int(kv["n"][0])
    ptr = np.array(kv["row_ptr"], np.int32)
    col = np.array(kv["col_idx"], np.int32)
    val = np.array(kv["val"], np.float64)
    X = np.array(kv["spmm_X"], np.float64).reshape(n, 2)
    want = np.array(kv["spmm_Y_a1_b0"], np.float64).reshape(m, 2)
    Y, _ = oracle.spmm_csr(m, n, ptr, col, val, X)
    assert np.array_equal(Y, want)


@pytest.mark.parametrize("k", [1, 3, 8])
def test_exact_rational(oracle_lib, k):
    """Every entry against the exact sum in rationals: within one rounding."""
    rng = np.random.default_rng(5 + k)
    A, dense = _random_csr(rng, 9, 7, 0.5)
    X = rng.uniform(-1, 1, (7, k))
    Yi = rng.uniform(-1, 1, (9, k))
    a, b = 1.5, -0.75
    Y, _ = oracle.spmm_csr(9, 7, A.indptr, A.indices, A.data, X, a, b, Yi)
    for i in range(9):
        for t in range(k):
            s = sum((Fraction(float(dense[i, j])) * Fraction(float(X[j, t])) for j in range(7)),
                    Fraction(0))
            exact = Fraction(a) * s + Fraction(b) * Fraction(float(Yi[i, t]))
            assert abs(Fraction(float(Y[i, t])) - exact) <= abs(exact) * Fraction(EPS), (i, t)


@pytest.mark.parametrize("k", [1, 2, 5, 16])
def test_dense_product(oracle_lib, k):
    rng = np.random.default_rng(100 + k)
    m, n = 60, 45
    A, dense = _random_csr(rng, m, n, 0.2)
    X = rng.standard_normal((n, k))
    Yi = rng.standard_normal((m, k))
    Y, S = oracle.spmm_csr(m, n, A.indptr, A.indices, A.data, X, 2.0, 0.5, Yi)
    want = 2.0 * (dense @ X) + 0.5 * Yi
    scale = 2.0 * (np.abs(dense) @ np.abs(X)) + 0.5 * np.abs(Yi)
    assert np.all(np.abs(Y - want) <= 4 * n * EPS * scale + 1e-300)
    assert np.allclose(S, scale, rtol=1e-12, atol=0)
    # beta = 0 never reads Y_in: NaN there changes nothing
    Y0, _ = oracle.spmm_csr(m, n, A.indptr, A.indices, A.data, X, 1.0, 0.0, None)
    assert np.all(np.abs(Y0 - dense @ X) <= 4 * n * EPS * (np.abs(dense) @ np.abs(X)) + 1e-300)


def test_columns_are_not_mixed(oracle_lib):
    """A transposed or shifted column index would mix columns: with X a
    one-hot block (column t is e_t), Y's column t must be A's column t."""
    rng = np.random.default_rng(9)
    A, dense = _random_csr(rng, 30, 6, 0.5)
    X = np.eye(6)
    Y, _ = oracle.spmm_csr(30, 6, A.indptr, A.indices, A.data, X)
    assert np.array_equal(Y, dense)


def test_stencil_times_constant_columns(oracle_lib):
    """7-point stencil times column t = (t+1)*ones: (t+1)*(6 - in-grid
    neighbours), exact."""
    A, _ = synth.stencil7_csr(12, seed=0)
    g = 12
    k = 4
    X = np.repeat(np.arange(1, k + 1, dtype=np.float64)[None, :], A.n, axis=0)
    Y, _ = oracle.spmm_csr(A.m, A.n, A.ptr, A.col, A.val, X)
    r = np.arange(A.m)
    base = np.zeros(A.m)
    for c in (r % g, (r // g) % g, r // (g * g)):
        base += (c == 0).astype(np.float64) + (c == g - 1).astype(np.float64)
    assert np.array_equal(Y, base[:, None] * np.arange(1, k + 1)[None, :])


def test_empty_and_argument_errors(oracle_lib):
    ptr = np.array([0, 0, 0], np.int32)
    Y, S = oracle.spmm_csr(2, 3, ptr, np.zeros(0, np.int32), np.zeros(0), np.ones((3, 2)),
                           1.0, 2.0, np.full((2, 2), 3.0))
    assert np.array_equal(Y, np.full((2, 2), 6.0))
    Y, _ = oracle.spmm_csr(2, 3, ptr, np.zeros(0, np.int32), np.zeros(0), np.ones((3, 0)))
    assert Y.shape == (2, 0)
    with pytest.raises(ValueError):
        oracle.spmm_csr(2, 3, ptr, np.zeros(0, np.int32), np.zeros(0), np.ones((4, 2)))


def test_leading_dimensions_wider_than_k(oracle_lib):
    """The C routine with ldx, ldy > k: NaN in the columns past k of X must
    not reach Y, Y's columns past k stay as they were, and columns < k equal
    the dense product."""
    import ctypes
    rng = np.random.default_rng(12)
    A, dense = _random_csr(rng, 20, 15, 0.3)
    k, ldx, ldy = 3, 5, 7
    X = np.full((15, ldx), np.nan)
    X[:, :k] = rng.uniform(-1, 1, (15, k))
    Y = np.full((20, ldy), 4.0)
    lib = oracle._load()
    ptr = np.ascontiguousarray(A.indptr, np.int32)
    col = np.ascontiguousarray(A.indices, np.int32)
    val = np.ascontiguousarray(A.data, np.float64)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    rc = lib.oracle_spmm_csr(20, 15, k, p(ptr), p(col), p(val), p(X), ldx, 1.0, 0.0, None, ldy,
                             p(Y), None)
    assert rc == 0
    assert np.all(Y[:, k:] == 4.0)
    want = dense @ X[:, :k]
    assert np.all(np.abs(Y[:, :k] - want) <= 4 * 15 * EPS * (np.abs(dense) @ np.abs(X[:, :k])) + 1e-300)
    assert lib.oracle_spmm_csr(20, 15, k, p(ptr), p(col), p(val), p(X), 2, 1.0, 0.0, None, ldy,
                               p(Y), None) == oracle.ERR_ARG
