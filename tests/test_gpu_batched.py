"""GPU parity of msrep_spmv_batched: every matrix of an uneven batch
(uniform and power-law, row counts log-uniform) against the oracle, across
repeated launches of the captured graph with fresh x/y pointers, and the
batched result equal to the single-matrix path on the same partitions."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import F32_TOL, F64_TOL, assert_close, stored_values

torch = pytest.importorskip("torch")
pk = pytest.importorskip("paper_2209_07552_amd")

pytestmark = pytest.mark.gpu


def _batch(count, m_hi, seed=0):
    return synth.batched_set(count, seed=seed, m_lo=100, m_hi=m_hi)


@pytest.mark.parametrize("vt", [0, 1])
@pytest.mark.parametrize("npw", [256, 1024, 4096])
def test_batched_parity(vt, npw):
    dev = torch.device("cuda:0")
    mats = _batch(24, 20_000, seed=1)
    Ms, v64s = [], []
    for A, _ in mats:
        sv, v64 = stored_values(A.val, vt)
        Ms.append(pk.Mat(pk.CSR, vt, A.m, A.n, ptr=A.ptr, idx=A.col, val=sv))
        v64s.append(v64)
    tunes = [pk.Tune(nnz_per_wave=npw) for _ in mats]
    alpha, beta = 1.5, -0.25
    plan = pk.msrep_plan_create(Ms, tunes, alpha, beta)
    assert plan.items() == sum(max(1, -(-A.nnz // npw)) for A, _ in mats)
    rng = np.random.default_rng(7)
    xdt = np.float64 if vt == 0 else np.float32
    tol = F64_TOL if vt == 0 else F32_TOL
    for rep in range(3):  # fresh x and y buffers every launch
        xs = [rng.uniform(-1, 1, A.n).astype(xdt) for A, _ in mats]
        yin = [rng.uniform(-1, 1, A.m).astype(xdt) for A, _ in mats]
        xd = [torch.from_numpy(x).to(dev) for x in xs]
        yd = [torch.from_numpy(y.copy()).to(dev) for y in yin]
        pk.msrep_spmv_batched(plan, xd, yd)
        torch.cuda.synchronize()
        for k, (A, _) in enumerate(mats):
            ref, s = oracle.spmv_csr(A.m, A.n, A.ptr, A.col, v64s[k], xs[k].astype(np.float64),
                                     alpha, beta, yin[k].astype(np.float64))
            assert_close(yd[k].cpu().numpy(), ref, s, tol, "batch rep%d matrix %d" % (rep, k))
    plan.destroy()


def test_batched_equals_single_path():
    dev = torch.device("cuda:0")
    mats = _batch(12, 50_000, seed=2)
    Ms = [pk.Mat(pk.CSR, pk.F64, A.m, A.n, ptr=A.ptr, idx=A.col, val=A.val) for A, _ in mats]
    plan = pk.msrep_plan_create(Ms, [pk.Tune(nnz_per_wave=512)] * len(Ms))
    xd = [torch.from_numpy(x).to(dev) for _, x in mats]
    yb = [torch.empty(A.m, dtype=torch.float64, device=dev) for A, _ in mats]
    pk.msrep_spmv_batched(plan, xd, yb)
    for k, (A, _) in enumerate(mats):
        P = pk.msrep_build_partition(Ms[k], max(1, -(-A.nnz // 512)))
        ys = torch.empty(A.m, dtype=torch.float64, device=dev)
        pk.msrep_spmv(Ms[k], P, xd[k], ys)
        torch.cuda.synchronize()
        assert torch.equal(yb[k], ys), k  # same partitions, same order: bit-identical


def test_batched_rejects_mixed_types():
    A, _ = synth.uniform_csr(100, 100, 5, seed=1)
    M0 = pk.Mat(pk.CSR, pk.F64, A.m, A.n, ptr=A.ptr, idx=A.col, val=A.val)
    M1 = pk.Mat(pk.CSR, pk.F32, A.m, A.n, ptr=A.ptr, idx=A.col, val=A.val.astype(np.float32))
    with pytest.raises(pk.MsrepError):
        pk.msrep_plan_create([M0, M1])


_full = {}


def _full_set():
    """The benchmark's batched set: 512 matrices, rows log-uniform in
    [1e3, 2e5], half uniform (4-64 per row) and half R-MAT-like."""
    if "mats" not in _full:
        _full["mats"] = synth.batched_set(512, seed=0)
    return _full["mats"]


@pytest.mark.slow
@pytest.mark.parametrize("vt,pf", [(0, 1), (1, 1), (0, 2)])
def test_batched_full_set_every_matrix(vt, pf):
    """All 512 matrices of the benchmark's set (416.7M nonzeros) in one plan,
    with the benchmark's launch shape and both load depths: every entry of
    every y against the oracle (FP32 values: on the stored values and
    FP32-rounded x)."""
    dev = torch.device("cuda:0")
    mats = _full_set()
    xdt = np.float64 if vt == 0 else np.float32
    Ms, xs, ys = [], [], []
    for A, x in mats:
        sv, _ = stored_values(A.val, vt)
        Ms.append(pk.Mat(pk.CSR, vt, A.m, A.n, ptr=A.ptr, idx=A.col, val=sv))
        xs.append(torch.from_numpy(x.astype(xdt)).to(dev))
        ys.append(torch.full((A.m,), float("nan"), dtype=xs[-1].dtype, device=dev))
    tunes = [pk.Tune(k_per_lane=4, waves_per_wg=4, nnz_per_wave=1024, pipeline=pf)] * len(Ms)
    plan = pk.msrep_plan_create(Ms, tunes)
    pk.msrep_spmv_batched(plan, xs, ys)
    torch.cuda.synchronize()
    tol = F64_TOL if vt == 0 else F32_TOL
    for k, (A, x) in enumerate(mats):
        v = A.val if vt == 0 else A.val.astype(np.float32).astype(np.float64)
        xo = x if vt == 0 else x.astype(np.float32).astype(np.float64)
        ref, s = oracle.spmv_csr(A.m, A.n, A.ptr, A.col, v, xo)
        assert_close(ys[k].cpu().numpy(), ref, s, tol, "full set vt%d pf%d matrix %d" % (vt, pf, k))
    plan.destroy()
    del Ms, xs, ys
    torch.cuda.empty_cache()


@pytest.mark.parametrize("count", [1, 3, 9, 40])
def test_batched_tiny_plans(count):
    """Plans whose grid has fewer workgroups than the GPU has XCDs (one item
    group per workgroup) and just above: every matrix against the oracle."""
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(count)
    mats = []
    for _ in range(count):
        m, n = int(rng.integers(1, 300)), int(rng.integers(1, 300))
        mats.append(synth.uniform_csr(m, n, min(3, n), seed=int(rng.integers(1 << 30)))[0])
    Ms = [pk.Mat(pk.CSR, pk.F64, A.m, A.n, ptr=A.ptr, idx=A.col, val=A.val) for A in mats]
    plan = pk.msrep_plan_create(Ms, [pk.Tune(nnz_per_wave=1 << 20, waves_per_wg=4)] * count, 2.0)
    assert plan.items() == count
    xs = [rng.uniform(-1, 1, A.n) for A in mats]
    xd = [torch.from_numpy(x).to(dev) for x in xs]
    yd = [torch.full((A.m,), float("nan"), dtype=torch.float64, device=dev) for A in mats]
    pk.msrep_spmv_batched(plan, xd, yd)
    torch.cuda.synchronize()
    for k, A in enumerate(mats):
        ref, s = oracle.spmv_csr(A.m, A.n, A.ptr, A.col, A.val, xs[k], 2.0)
        assert_close(yd[k].cpu().numpy(), ref, s, F64_TOL, "tiny plan %d matrix %d" % (count, k))
    plan.destroy()
