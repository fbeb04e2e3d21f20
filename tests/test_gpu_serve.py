"""GPU tests of msrep_serve: every request's last y against the oracle (x
regenerated from the published SplitMix64 definition on the host), the same
result alone and in the mix (bit-identical), and admission that binds under
a small budget."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import F32_TOL, F64_TOL, assert_close

torch = pytest.importorskip("torch")
pk = pytest.importorskip("paper_2209_07552_amd")
from paper_2209_07552_amd import serving  # noqa: E402

pytestmark = pytest.mark.gpu

SEED = 1234


def _pool(count=6, m_hi=30_000):
    return [A for A, _ in synth.batched_set(count, seed=8, m_lo=500, m_hi=m_hi)]


def _check_last_y(pool, trace, res, vt):
    tol = F64_TOL if vt == pk.F64 else F32_TOL
    for q, r in zip(trace, res):
        assert r.status == 0, q
        A = pool[q.matrix]
        x = synth.serving_x(A.n, SEED, q.rid, q.steps - 1)
        val = A.val
        if vt == pk.F32:
            x = x.astype(np.float32).astype(np.float64)
            val = A.val.astype(np.float32).astype(np.float64)
        ref, s = oracle.spmv_csr(A.m, A.n, A.ptr, A.col, val, x)
        assert_close(r.y, ref, s, tol, "request %d" % q.rid)


@pytest.mark.parametrize("vt", [0, 1])
def test_serve_results_match_oracle(vt):
    pool = _pool()
    trace = synth.serving_trace(24, rate=20000.0, pool=len(pool), seed=3, k_lo=2, k_hi=8)
    res, st = serving.serve(pool, trace, budget_bytes=2 << 30, vtype=vt, seed=SEED, keep_y=True)
    assert st["n_done"] == len(trace) and st["ticks"] > 0
    _check_last_y(pool, trace, res, vt)


def test_alone_equals_mix():
    pool = _pool()
    trace = synth.serving_trace(16, rate=1e6, pool=len(pool), seed=6, k_lo=3, k_hi=7)
    mix, st = serving.serve(pool, trace, budget_bytes=2 << 30, seed=SEED, keep_y=True)
    assert st["peak_active"] > 1  # requests really ran together
    for q, r in zip(trace[:6], mix[:6]):
        alone, _ = serving.serve(pool, [synth.Request(q.rid, 0.0, q.matrix, q.steps)],
                                 budget_bytes=2 << 30, seed=SEED, keep_y=True)
        assert np.array_equal(alone[0].y, r.y), q.rid


def test_small_budget_queues():
    pool = _pool(4, m_hi=20_000)
    trace = synth.serving_trace(12, rate=1e6, pool=len(pool), seed=7, k_lo=2, k_hi=4)
    # tick tables + room for roughly one request at a time
    budget = 24 << 20
    res, st = serving.serve(pool, trace, budget_bytes=budget, max_slots=8, seed=SEED, keep_y=True)
    assert st["peak_bytes"] <= budget
    ok = [r.status == 0 for r in res]
    assert any(ok)
    _check_last_y(pool, [q for q, o in zip(trace, ok) if o], [r for r, o in zip(res, ok) if o], 0)


@pytest.mark.parametrize("vt", [0, 1])
def test_fill_x_matches_published_generator(vt):
    """The device x generator (msrep_serve_fill_x, also the server's) equals
    the host's SplitMix64 values, rounded once to FP32 for F32."""
    n = 100_003
    dt = torch.float64 if vt == pk.F64 else torch.float32
    for rid, step in ((0, 0), (7, 3), ((1 << 24) - 1, 65535)):
        x = torch.full((n,), float("nan"), dtype=dt, device="cuda")
        serving.fill_x(x, SEED, rid, step)
        torch.cuda.synchronize()
        want = synth.serving_x(n, SEED, rid, step)
        if vt == pk.F32:
            want = want.astype(np.float32)
        assert np.array_equal(x.cpu().numpy(), want), (rid, step)
