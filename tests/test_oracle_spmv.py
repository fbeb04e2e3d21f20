"""Pins for the oracle's SpMV (Sec. 2.2, Algorithm 1): exact rational sums,
dense products, scipy, closed forms and a hand-worked example.  None of these
compares the oracle with itself."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from conftest import load_golden

EPS = np.finfo(np.float64).eps


def _random_csr(rng, m, n, density, empty_rows=True):
    dense = rng.uniform(-1, 1, (m, n)) * (rng.random((m, n)) < density)
    if empty_rows and m > 2:
        dense[rng.integers(0, m, size=max(1, m // 4))] = 0.0
    A = sp.csr_matrix(dense)
    A.sort_indices()
    return A, dense


def _fmts(A):
    """The same matrix as (csr, csc, coo) arrays via scipy (a library
    reduction with a unique answer)."""
    C = A.tocsc()
    C.sort_indices()
    O = A.tocoo()
    return C, O


def _all_formats(m, n, A, x, alpha=1.0, beta=0.0, y_in=None):
    C, O = _fmts(A)
    r = oracle.spmv_csr(m, n, A.indptr, A.indices, A.data, x, alpha, beta, y_in)
    c = oracle.spmv_csc(m, n, C.indptr, C.indices, C.data, x, alpha, beta, y_in)
    o = oracle.spmv_coo(m, n, O.row, O.col, O.data, x, alpha, beta, y_in)
    return r, c, o


def test_golden_example(oracle_lib):
    kv, _ = load_golden("example_6x6.txt")
    m, n = int(kv["m"][0]), int(kv["n"][0])
    ptr = np.array(kv["row_ptr"], np.int32)
    col = np.array(kv["col_idx"], np.int32)
    val = np.array(kv["val"], np.float64)
    x = np.array(kv["x"], np.float64)
    y0 = np.array(kv["y_a1_b0"], np.float64)
    y2 = np.array(kv["y_a2_bm1"], np.float64)
    yin = np.array(kv["y_in"], np.float64)
    cptr = np.array(kv["csc_col_ptr"], np.int32)
    crow = np.array(kv["csc_row_idx"], np.int32)
    cval = np.array(kv["csc_val"], np.float64)
    orow = np.array(kv["coo_row_idx"], np.int32)
    for a, b, yi, want in ((1.0, 0.0, None, y0), (2.0, -1.0, yin, y2)):
        y, _ = oracle.spmv_csr(m, n, ptr, col, val, x, a, b, yi)
        assert np.array_equal(y, want)
        y, _ = oracle.spmv_csc(m, n, cptr, crow, cval, x, a, b, yi)
        assert np.array_equal(y, want)
        y, _ = oracle.spmv_coo(m, n, orow, col, val, x, a, b, yi)
        assert np.array_equal(y, want)


@pytest.mark.parametrize("seed", range(12))
def test_exact_rational(oracle_lib, seed):
    """Dot2 result against the exact rational value: within one rounding of
    the exact sum (plus the Dot2 second-order term)."""
    rng = np.random.default_rng(seed)
    m, n = int(rng.integers(1, 14)), int(rng.integers(1, 14))
    A, dense = _random_csr(rng, m, n, 0.5)
    # wide dynamic range and cancellation-prone values
    x = rng.uniform(-1, 1, n) * 10.0 ** rng.integers(-8, 9, n)
    alpha, beta = float(rng.uniform(-3, 3)), float(rng.choice([0.0, rng.uniform(-2, 2)]))
    y_in = rng.uniform(-1, 1, m)
    exact, absolute = [], []
    for i in range(m):
        a = sum((abs(Fraction(dense[i, j]) * Fraction(x[j])) for j in range(n)), Fraction(0))
        a = abs(Fraction(alpha)) * a + (abs(Fraction(beta) * Fraction(y_in[i])) if beta else 0)
        absolute.append(a)
        s = sum((Fraction(dense[i, j]) * Fraction(x[j]) for j in range(n)), Fraction(0))
        e = Fraction(alpha) * s
        if beta != 0.0:
            e += Fraction(beta) * Fraction(y_in[i])
        exact.append(e)
    for y, s in _all_formats(m, n, A, x, alpha, beta, y_in):
        for i in range(m):
            err = abs(Fraction(y[i]) - exact[i])
            bound = Fraction(EPS) * abs(exact[i]) + Fraction(1e-28) * Fraction(s[i])
            assert err <= bound, (i, float(err), float(bound))
            # the tolerance scale |alpha|(|A||x|)_i + |beta||y_i|, to n*u
            assert abs(Fraction(s[i]) - absolute[i]) <= Fraction(32 * EPS) * absolute[i]


def test_dense_numpy(oracle_lib):
    rng = np.random.default_rng(7)
    m, n = 64, 48
    A, dense = _random_csr(rng, m, n, 0.3)
    x = rng.uniform(-1, 1, n)
    ref = dense @ x
    for y, s in _all_formats(m, n, A, x):
        assert np.all(np.abs(y - ref) <= 64 * EPS * s + 1e-300)
        assert np.allclose(s, np.abs(dense) @ np.abs(x), rtol=1e-13, atol=0)


def test_uniform_4096_vs_scipy(oracle_lib):
    A, x = synth.uniform_csr(4096, 4096, 16, seed=0)
    S = sp.csr_matrix((A.val, A.col, A.ptr), shape=(A.m, A.n))
    ref = S @ x
    y, s = oracle.spmv_csr(A.m, A.n, A.ptr, A.col, A.val, x)
    assert np.all(np.abs(y - ref) <= 32 * EPS * s)
    assert np.allclose(s, abs(S) @ np.abs(x), rtol=1e-13)


def test_identity_permutation_diagonal(oracle_lib):
    rng = np.random.default_rng(3)
    n = 257
    x = rng.uniform(-1, 1, n) * 10.0 ** rng.integers(-20, 20, n)
    eye = sp.identity(n, format="csr")
    for y, _ in _all_formats(n, n, eye, x):
        assert np.array_equal(y, x)
    perm = rng.permutation(n)
    P = sp.csr_matrix((np.ones(n), (np.arange(n), perm)), shape=(n, n))
    for y, _ in _all_formats(n, n, P, x):
        assert np.array_equal(y, x[perm])
    d = rng.uniform(-5, 5, n)
    D = sp.diags(d, format="csr")
    for y, _ in _all_formats(n, n, D, x):
        assert np.array_equal(y, d * x)  # one correctly rounded product each


@pytest.mark.parametrize("g", [1, 2, 5, 16])
def test_stencil_times_ones(oracle_lib, g):
    """7-point Laplacian times ones = number of missing neighbours."""
    A, _ = synth.stencil7_csr(g)
    y, _ = oracle.spmv_csr(A.m, A.n, A.ptr, A.col, A.val, np.ones(A.n))
    r = np.arange(A.m)
    i, j, k = r % g, (r // g) % g, r // (g * g)
    missing = sum(((c == 0).astype(int) + (c == g - 1).astype(int)) for c in (i, j, k))
    assert np.array_equal(y, missing.astype(np.float64))


def test_dyadic_exact(oracle_lib):
    """Dyadic values and x: every product and partial sum is exact, so the
    result equals the integer sum scaled by 2^-16."""
    rng = np.random.default_rng(11)
    A, _ = synth.uniform_csr(300, 200, 40, seed=5)
    A.val = synth.dyadic(rng, A.nnz)
    x = synth.dyadic(rng, A.n)
    iv = np.rint(A.val * 256).astype(np.int64)
    ix = np.rint(x * 256).astype(np.int64)
    want = np.zeros(A.m)
    for r in range(A.m):
        a, b = A.ptr[r], A.ptr[r + 1]
        want[r] = int(np.sum(iv[a:b] * ix[A.col[a:b]])) / 65536.0
    S = sp.csr_matrix((A.val, A.col, A.ptr), shape=(A.m, A.n))
    for y, _ in _all_formats(A.m, A.n, S, x):
        assert np.array_equal(y, want)


def test_beta_zero_ignores_y_and_nan_propagates(oracle_lib):
    ptr = np.array([0, 1, 2], np.int32)
    col = np.array([0, 1], np.int32)
    val = np.array([2.0, 3.0])
    x = np.array([1.0, np.nan])
    y_in = np.array([np.nan, np.nan])
    y, _ = oracle.spmv_csr(2, 2, ptr, col, val, x, 1.0, 0.0, y_in)
    assert y[0] == 2.0 and np.isnan(y[1])
    y, _ = oracle.spmv_csr(2, 2, ptr, col, val, np.array([1.0, 1.0]), 1.0, 0.5, y_in)
    assert np.isnan(y[0]) and np.isnan(y[1])


def test_empty_matrix(oracle_lib):
    ptr = np.zeros(4, np.int32)
    y, s = oracle.spmv_csr(3, 5, ptr, np.zeros(0, np.int32), np.zeros(0), np.ones(5),
                           1.0, 2.0, np.array([1.0, -2.0, 0.5]))
    assert np.array_equal(y, [2.0, -4.0, 1.0])
    assert np.array_equal(s, [2.0, 4.0, 1.0])


def test_rejects_bad_index(oracle_lib):
    ptr = np.array([0, 1], np.int32)
    with pytest.raises(ValueError):
        oracle.spmv_csr(1, 2, ptr, np.array([5], np.int32), np.ones(1), np.ones(2))
