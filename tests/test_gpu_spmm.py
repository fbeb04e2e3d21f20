"""GPU parity of msrep_spmm (k right-hand sides over the CSR partitions)
against the oracle's per-column product: FP64 within 1e-12 and FP32 / BF16
values within 1e-5 of |alpha||A||X| + |beta||Y| per entry, bit-exact on
dyadic inputs and on the stencil times constant columns, columns beyond k
untouched, and every pass width (8, 4, 2, 1 columns) and partition count
from one to more partitions than nonzeros.  Every call goes through the C
ABI."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import F32_TOL, F64_TOL, assert_close, stored_values

torch = pytest.importorskip("torch")
pk = pytest.importorskip("paper_2209_07552_amd")

pytestmark = pytest.mark.gpu


def _dev():
    return torch.device("cuda:0")


def _mk(rng, counts, n, name):
    counts = np.asarray(counts, np.int64)
    cols = np.concatenate([np.sort(rng.choice(n, c, replace=False)) for c in counts]) \
        if counts.sum() else np.zeros(0, np.int64)
    ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    return synth.Csr(len(counts), n, ptr, cols.astype(np.int32),
                     rng.uniform(-1, 1, int(counts.sum())), name=name)


def _matrices():
    rng = np.random.default_rng(17)
    out = [
        _mk(rng, [0, 0, 0], 5, "all-empty"),
        _mk(rng, [7], 9, "one-row"),
        _mk(rng, [0, 0, 3000, 0, 1, 0, 0], 4000, "long-row"),
        _mk(rng, [0] * 50 + [2] * 10 + [0] * 40, 64, "lead-trail-empty"),
        _mk(rng, rng.integers(0, 40, 300) * (rng.random(300) < 0.5), 200, "ragged"),
        _mk(rng, [0] * 3000 + [1, 0, 0, 2] * 500 + [0] * 2000, 50, "sparse-runs"),
    ]
    A, _ = synth.rmat_csr(scale=11, edge_factor=8, seed=3)
    out.append(A)
    A, _ = synth.stencil7_csr(10, seed=0)
    out.append(A)
    return out


def _run(A, vt, k, np_, alpha=1.0, beta=0.0, ld_extra=0, seed=0, X64=None, val=None):
    """Device SpMM and the oracle's result for the stored values."""
    rng = np.random.default_rng(seed)
    v = A.val if val is None else val
    sv, v64 = stored_values(v, vt)
    M = pk.Mat(pk.CSR, vt, A.m, A.n, ptr=A.ptr, idx=A.col, val=sv)
    P = pk.msrep_build_partition(M, np_)
    tdt = torch.float64 if vt == pk.F64 else torch.float32
    ndt = np.float64 if vt == pk.F64 else np.float32
    if X64 is None:
        X64 = rng.uniform(-1, 1, (A.n, k))
    Xh = X64.astype(ndt)
    Yin = rng.uniform(-1, 1, (A.m, k)).astype(ndt)
    ldx, ldy = k + ld_extra, k + ld_extra
    Xw = np.full((A.n, ldx), np.nan, ndt)
    Xw[:, :k] = Xh
    Yw = np.full((A.m, ldy), 7.0, ndt)
    Yw[:, :k] = Yin if beta != 0.0 else np.nan
    Xd = torch.from_numpy(Xw).to(_dev())[:, :k]
    Yd_full = torch.from_numpy(Yw).to(_dev())
    Yd = Yd_full[:, :k]
    pk.msrep_spmm(M, P, Xd, Yd, alpha, beta)
    torch.cuda.synchronize()
    out = Yd_full.cpu().numpy()
    ref, s = oracle.spmm_csr(A.m, A.n, A.ptr, A.col, v64, Xh.astype(np.float64), alpha, beta,
                             Yin.astype(np.float64) if beta != 0.0 else None)
    if ld_extra:
        assert np.all(out[:, k:] == 7.0), "columns beyond k were written"
    return out[:, :k].astype(np.float64), ref, s


def _check(A, vt, k, np_, **kw):
    y, ref, s = _run(A, vt, k, np_, **kw)
    tol = F64_TOL if vt == pk.F64 else F32_TOL
    what = "%s vt%d k%d np%d" % (A.name, vt, k, np_)
    assert_close(y.ravel(), ref.ravel(), s.ravel(), tol, what)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 12, 17])
def test_spmm_columns_fp64(k):
    for A in _matrices():
        for np_ in (1, 3, max(1, A.nnz // 97), max(1, A.nnz // 16)):
            _check(A, pk.F64, k, np_, seed=k)


@pytest.mark.parametrize("vt", [1, 2])
@pytest.mark.parametrize("k", [4, 8, 11])
def test_spmm_low_precision_values(vt, k):
    for A in _matrices():
        _check(A, vt, k, max(1, A.nnz // 64), seed=k + 10 * vt)


@pytest.mark.parametrize("vt", [0, 1])
def test_spmm_alpha_beta_and_leading_dimension(vt):
    for A in _matrices():
        for k in (3, 8, 9):
            _check(A, vt, k, max(1, A.nnz // 50), alpha=-1.25, beta=0.5, ld_extra=5, seed=k)
            _check(A, vt, k, max(1, A.nnz // 50), alpha=2.0, beta=0.0, ld_extra=3, seed=k + 1)


def test_spmm_more_partitions_than_nonzeros():
    rng = np.random.default_rng(2)
    A = _mk(rng, [0, 3, 0, 0, 2, 0], 8, "tiny")
    for np_ in (5, 6, 9, 40):
        _check(A, pk.F64, 8, np_, beta=1.5, seed=np_)


def test_spmm_dyadic_bit_exact():
    """Dyadic values and X: every partial sum is exact, so the result must
    equal the oracle's bit for bit (pins the row split, the carries between
    chunks and the boundary merge of every column)."""
    rng = np.random.default_rng(41)
    for A in _matrices():
        val = synth.dyadic(rng, A.nnz)
        X = synth.dyadic(rng, A.n * 12).reshape(A.n, 12)
        for np_ in (1, max(1, A.nnz // 100), max(1, A.nnz // 7)):
            y, ref, _ = _run(A, pk.F64, 12, np_, X64=X, val=val)
            assert np.array_equal(y, ref), (A.name, np_, int(np.sum(y != ref)))


@pytest.mark.parametrize("vt", [0, 1])
def test_spmm_column_pairs_and_single_columns(vt):
    """Eight columns run two per lane when X and Y rows keep column pairs
    aligned (even leading dimensions) and one per lane otherwise; both
    layouts must give the oracle's result (dyadic inputs: bit for bit)."""
    rng = np.random.default_rng(77)
    A, _ = synth.rmat_csr(scale=11, edge_factor=8, seed=4)
    val = synth.dyadic(rng, A.nnz)
    X = synth.dyadic(rng, A.n * 8).reshape(A.n, 8)
    for extra in (0, 1, 2, 3):  # ldx = ldy = 8, 9, 10, 11
        y, ref, s = _run(A, vt, 8, max(1, A.nnz // 300), X64=X, val=val, ld_extra=extra,
                         alpha=0.5, beta=0.25 if extra % 2 else 0.0, seed=extra)
        if vt == pk.F64:
            assert np.array_equal(y, ref), (extra, int(np.sum(y != ref)))
        else:
            assert_close(y.ravel(), ref.ravel(), s.ravel(), F32_TOL, "ld %d" % (8 + extra))


def test_spmm_columns_match_spmv():
    """Column j of msrep_spmm equals msrep_spmv with x = X[:, j] (dyadic, so
    both are exact and must agree bit for bit)."""
    rng = np.random.default_rng(8)
    A, _ = synth.rmat_csr(scale=12, edge_factor=8, seed=1)
    val = synth.dyadic(rng, A.nnz)
    X = synth.dyadic(rng, A.n * 5).reshape(A.n, 5)
    M = pk.Mat(pk.CSR, pk.F64, A.m, A.n, ptr=A.ptr, idx=A.col, val=val)
    P = pk.msrep_build_partition(M, A.nnz // 256)
    Xd = torch.from_numpy(X).to(_dev())
    Yd = torch.empty((A.m, 5), dtype=torch.float64, device=_dev())
    pk.msrep_spmm(M, P, Xd, Yd)
    for j in range(5):
        y = torch.empty(A.m, dtype=torch.float64, device=_dev())
        pk.msrep_spmv(M, P, Xd[:, j].contiguous(), y)
        assert torch.equal(y, Yd[:, j]), j


@pytest.mark.slow
@pytest.mark.parametrize("vt", [0, 1, 2])
def test_spmm_stencil_full_size_exact(vt):
    """256^3 stencil (16.7M rows) times column t = t+1: (t+1)*(6 - in-grid
    neighbours), exact in every value type (6 and -1 and the small integer
    results are exact in BF16 and FP32), at the partition size the benchmark
    uses."""
    A, _ = synth.stencil7_csr(256, seed=0)
    k = 8
    sv, _ = stored_values(A.val, vt)
    M = pk.Mat(pk.CSR, vt, A.m, A.n, ptr=A.ptr, idx=A.col, val=sv)
    P = pk.msrep_build_partition(M, -(-A.nnz // 2048))
    dt = torch.float64 if vt == pk.F64 else torch.float32
    Xd = torch.arange(1, k + 1, dtype=dt, device=_dev()).repeat(A.n, 1)
    Yd = torch.full((A.m, k), float("nan"), dtype=dt, device=_dev())
    pk.msrep_spmm(M, P, Xd, Yd)
    torch.cuda.synchronize()
    g = 256
    r = torch.arange(A.m, device=_dev())
    base = torch.zeros(A.m, dtype=dt, device=_dev())
    for c in (r % g, (r // g) % g, r // (g * g)):
        base += (c == 0).to(dt) + (c == g - 1).to(dt)
    want = base[:, None] * torch.arange(1, k + 1, dtype=dt, device=_dev())[None, :]
    assert torch.equal(Yd, want), vt
    del M, P, Xd, Yd, want, base, r
    torch.cuda.empty_cache()


@pytest.mark.slow
def test_spmm_rmat_full_size():
    """R-MAT scale 20 with k = 8 at the benchmark's partition size against the
    oracle, every entry."""
    A, _ = synth.rmat_csr(scale=20, edge_factor=16, seed=0)
    _check(A, pk.F64, 8, -(-A.nnz // 512), seed=3)
    del A
    torch.cuda.empty_cache()


@pytest.mark.parametrize("k", [8, 5])
def test_spmm_replays_under_graph_capture(k):
    """msrep_spmm launches kernels only (no memsets, no allocation when the
    workspace is passed), so a caller can capture it: three replays with new
    X contents, eager work and synchronisation in between, each equal to the
    eager call on the same X and within tolerance of the oracle."""
    A, _ = synth.rmat_csr(scale=13, edge_factor=8, seed=23)
    M = pk.Mat(pk.CSR, pk.F64, A.m, A.n, ptr=A.ptr, idx=A.col, val=A.val)
    P = pk.msrep_build_partition(M, 300)
    dev = _dev()
    X = torch.zeros((A.n, k), dtype=torch.float64, device=dev)
    Y = torch.zeros((A.m, k), dtype=torch.float64, device=dev)
    ws = torch.zeros(pk.msrep_spmm_ws_bytes(M, P.np, k), dtype=torch.uint8, device=dev)
    pk.msrep_spmm(M, P, X, Y, ws=ws)  # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pk.msrep_spmm(M, P, X, Y, ws=ws)
    rng = np.random.default_rng(24)
    for rep in range(3):
        Xn = rng.uniform(-1, 1, (A.n, k))
        X.copy_(torch.from_numpy(Xn))
        g.replay()
        torch.cuda.synchronize()
        got = Y.cpu().numpy().copy()
        Y_eager = torch.zeros_like(Y)
        pk.msrep_spmm(M, P, X, Y_eager, ws=torch.zeros_like(ws))
        torch.cuda.synchronize()
        ref, sc = oracle.spmm_csr(A.m, A.n, A.ptr, A.col, A.val, Xn)
        assert_close(got.ravel(), ref.ravel(), sc.ravel(), F64_TOL, "k%d replay %d" % (k, rep))
        assert np.array_equal(got, Y_eager.cpu().numpy()), (k, rep)


def test_spmm_errors():
    A = synth.stencil7_csr(4, seed=0)[0]
    M = pk.Mat(pk.CSR, pk.F64, A.m, A.n, ptr=A.ptr, idx=A.col, val=A.val)
    P = pk.msrep_build_partition(M, 4)
    X = torch.zeros((A.n, 3), dtype=torch.float64, device=_dev())
    Y = torch.zeros((A.m, 3), dtype=torch.float64, device=_dev())
    small = torch.empty(8, dtype=torch.uint8, device=_dev())
    with pytest.raises(pk.MsrepError):
        pk.msrep_spmm(M, P, X, Y, ws=small)
    H = oracle.transpose(A.m, A.n, A.ptr, A.col)
    C = pk.Mat(pk.CSC, pk.F64, A.m, A.n, ptr=H[0], idx=H[1], val=A.val[H[3]])
    PC = pk.msrep_build_partition(C, 4)
    with pytest.raises(pk.MsrepError):
        pk.msrep_spmm(C, PC, X, Y)
    pk.msrep_spmm(M, P, X[:, :0], Y[:, :0])  # k == 0: nothing to do
