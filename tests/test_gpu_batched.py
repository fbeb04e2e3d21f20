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
