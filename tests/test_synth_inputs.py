"""The synthetic inputs have the structure the workloads claim (CPU only):
R-MAT's column degrees follow a power law with exponent in the interval the
paper uses to pick its matrices (P(k) ~ k^-R, k = nonzeros per column,
R in [1, 4]); the 7-point stencil has the closed-form nonzero count and
entries; the batched set alternates uniform and R-MAT-like matrices with
row counts inside the stated range."""
import math

import numpy as np

import synth


def _mle_exponent(k, kmin):
    """Discrete power-law exponent by maximum likelihood over k >= kmin
    (the continuous estimator with the usual half-unit shift)."""
    kk = k[k >= kmin].astype(np.float64)
    return 1.0 + kk.size / np.sum(np.log(kk / (kmin - 0.5)))


def test_rmat_column_degrees_are_power_law():
    A, _ = synth.rmat_csr(16, seed=0)
    k = np.bincount(A.col, minlength=A.n)
    k = k[k > 0]
    for kmin in (8, 16, 32):
        R = _mle_exponent(k, kmin)
        assert 1.0 <= R <= 4.0, (kmin, R)
    assert k.max() > 100 * k.mean()  # a heavy tail: a few columns hold many nonzeros


def test_uniform_control_is_not_power_law():
    A, _ = synth.uniform_csr(65536, 65536, 16, seed=0)
    k = np.bincount(A.col, minlength=A.n)
    k = k[k > 0]
    assert k.max() < 3 * k.mean()
    assert _mle_exponent(k, 16) > 4.0


def test_stencil_structure():
    g = 16
    A, x = synth.stencil7_csr(g, seed=0)
    assert A.m == A.n == g ** 3 and A.nnz == 7 * g ** 3 - 6 * g ** 2
    rows = np.repeat(np.arange(A.m), np.diff(A.ptr))
    d = A.col.astype(np.int64) - rows
    assert set(np.unique(d)) == {-g * g, -g, -1, 0, 1, g, g * g}
    assert np.all(A.val[d == 0] == 6.0) and np.all(A.val[d != 0] == -1.0)
    # no wrap-around: a neighbour along an axis exists only inside the grid
    i, j, kz = rows % g, (rows // g) % g, rows // (g * g)
    assert np.all(i[d == 1] < g - 1) and np.all(i[d == -1] > 0)
    assert np.all(j[d == g] < g - 1) and np.all(kz[d == g * g] < g - 1)
    assert x.min() >= -1.0 and x.max() <= 1.0


def test_batched_set_shapes():
    count = 16
    mats = synth.batched_set(count, seed=0)
    for k, (A, _) in enumerate(mats):
        assert 1_000 <= A.m <= 200_000 and A.m == A.n
        assert A.name.endswith("uniform" if k % 2 == 0 else "rmat")
        deg = np.diff(A.ptr)
        if k % 2 == 0:
            assert deg.min() >= 4 and deg.max() <= 64
        assert np.all(np.diff(A.col[A.ptr[0]:A.ptr[1]]) > 0)  # sorted, distinct
    ms = np.array([A.m for A, _ in mats])
    assert math.log(ms.max() / ms.min()) > 1.0  # spread over the log-uniform range
