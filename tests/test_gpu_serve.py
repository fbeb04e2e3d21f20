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


@pytest.mark.parametrize("vt", [0, 1])
def test_steps_per_tick_same_results(vt):
    """A request's steps run several to a tick, as the columns of
    multi-vector passes (blocks of 8 columns, each one pass of 8 or passes of
    4, 2 and 1): the last y matches the oracle with 1, 3, 5, 8, 13 (a full
    block and a partial one) and 64 steps per tick; 1..40 steps per request
    leave partial groups of every size, and the last step lands in every
    column position and block.  From 8 steps per tick up, every tick but a
    request's last runs whole blocks of 8, so the results are bit-identical
    for 8, 13 and 64 (and whatever the load made each tick's cap)."""
    pool = _pool()
    trace = synth.serving_trace(20, rate=5e4, pool=len(pool), seed=9, k_lo=1, k_hi=40)
    outs = {}
    for spt in (1, 3, 5, 8, 13, 64):
        res, st = serving.serve(pool, trace, budget_bytes=2 << 30, vtype=vt, seed=SEED,
                                keep_y=True, steps_per_tick=spt)
        assert st["n_done"] == len(trace) and st["n_failed"] == 0
        _check_last_y(pool, trace, res, vt)
        outs[spt] = (res, st)
    # (how requests share ticks depends on timing; only bounds are fixed)
    ticks = {spt: st["ticks"] for spt, (_, st) in outs.items()}
    mx = max(q.steps for q in trace)
    assert ticks[1] >= mx and ticks[3] >= -(-mx // 3) and ticks[64] < ticks[1]
    for spt in (13, 64):
        for q, a, b in zip(trace, outs[8][0], outs[spt][0]):
            assert np.array_equal(a.y, b.y), (spt, q.rid)


def test_incremental_server_register():
    """msrep_server_register: matrices added to a running server's pool (from
    another host thread while requests run) get the next indices, and
    requests on them complete with the oracle's last y; a bad matrix is
    refused."""
    import ctypes
    import threading
    import time
    pool = _pool(3)
    extra = [A for A, _ in synth.batched_set(3, seed=21, m_lo=400, m_hi=12_000)]
    got, idx = {}, []
    with serving.Server(pool, 2 << 30, seed=SEED) as S:
        for rid in range(6):
            S.submit(rid, rid % 3, 4, keep_y=True)
        th = threading.Thread(target=lambda: idx.extend(S.register(A) for A in extra))
        th.start()
        th.join()
        assert idx == [3, 4, 5]
        reqs = [(rid, k, 3 + rid % 5) for rid, k in zip(range(6, 15), [3, 4, 5] * 3)]
        for rid, k, steps in reqs:
            S.submit(rid, k, steps, keep_y=True)
        with pytest.raises(pk.MsrepError):
            S.submit(99, 6, 2)  # no matrix 6 yet
        bad = synth.uniform_csr(10, 10, 2, seed=1)[0]
        hm, keep = serving._host_pool([bad], pk.F32, pinned=False)  # wrong value type
        i = ctypes.c_int32(-1)
        assert S._L.msrep_server_register(S._h, hm, ctypes.byref(i)) == -1 and i.value == -1
        deadline = time.time() + 60
        while len(got) < 15 and time.time() < deadline:
            for c in S.poll(timeout_ms=50):
                assert c.status == 0, c
                got[c.rid] = c
        assert len(got) == 15
        ys = {rid: S.y_of(rid).copy() for rid, _, _ in reqs}
        st = S.close()
    assert st["n_done"] == 15
    full = pool + extra
    for rid, k, steps in reqs:
        ref, sc = _oracle_y(full[k], rid, steps, pk.F64)
        assert_close(ys[rid], ref, sc, F64_TOL, "registered matrix %d, request %d" % (k, rid))


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


def test_small_arena_reserves_eight_columns_same_results():
    """With an arena too small for a request's full set of columns (more
    than a sixteenth of it), requests reserve 8 columns and run 8 steps a
    tick; since every tick but a request's last runs whole blocks of 8, the
    last y is bit-identical to a roomy arena's (all steps in one or two
    ticks), and matches the oracle."""
    # 15,000-20,000 rows: 17 or more steps reserve at least 24 columns, over
    # 5 MB of vectors, beyond a sixteenth of the small arena
    pool = [A for A, _ in synth.batched_set(3, seed=8, m_lo=15_000, m_hi=20_000)]
    trace = synth.serving_trace(8, rate=2e3, pool=len(pool), seed=12, k_lo=17, k_hi=40)
    big, st_big = serving.serve(pool, trace, budget_bytes=2 << 30, seed=SEED, keep_y=True)
    small, st_small = serving.serve(pool, trace, budget_bytes=48 << 20, seed=SEED, keep_y=True)
    assert all(r.status == 0 for r in big) and all(r.status == 0 for r in small)
    assert st_small["peak_bytes"] <= 48 << 20
    assert st_small["ticks"] > st_big["ticks"]  # 8 steps a tick against up to 64
    for q, a, b in zip(trace, big, small):
        assert np.array_equal(a.y, b.y), q.rid
    _check_last_y(pool, trace, small, 0)


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


def _oracle_y(A, rid, steps, vt):
    x = synth.serving_x(A.n, SEED, rid, steps - 1)
    val = A.val
    if vt == pk.F32:
        x = x.astype(np.float32).astype(np.float64)
        val = A.val.astype(np.float32).astype(np.float64)
    return oracle.spmv_csr(A.m, A.n, A.ptr, A.col, val, x)


@pytest.mark.parametrize("vt", [0, 1])
def test_incremental_server_results(vt):
    """msrep_server_*: requests submitted from two host threads while others
    run, completions polled as they come; every last y matches the oracle
    and equals the trace-replay server's y for the same request bit for
    bit; the statistics count every request."""
    import threading
    import time
    pool = _pool()
    reqs = [(rid, rid % len(pool), 2 + (rid * 7) % 9) for rid in range(24)]
    tol = F64_TOL if vt == pk.F64 else F32_TOL
    got = {}
    with serving.Server(pool, 2 << 30, vtype=vt, seed=SEED) as S:
        def feed(part):
            for rid, k, steps in part:
                S.submit(rid, k, steps, keep_y=True)
                time.sleep(0.0005)
        th = [threading.Thread(target=feed, args=(reqs[i::2],)) for i in range(2)]
        for t in th:
            t.start()
        deadline = time.time() + 60
        while len(got) < len(reqs) and time.time() < deadline:
            for c in S.poll(timeout_ms=50):
                assert c.status == 0, c
                assert c.t_arrive <= c.t_admit <= c.t_done, c
                got[c.rid] = c
        for t in th:
            t.join()
        assert len(got) == len(reqs)
        ys = {rid: S.y_of(rid).copy() for rid, _, _ in reqs}
        st = S.close()
    assert st["n_done"] == len(reqs) and st["n_failed"] == 0 and st["ticks"] > 0
    for rid, k, steps in reqs:
        ref, s = _oracle_y(pool[k], rid, steps, vt)
        assert_close(ys[rid], ref, s, tol, "server request %d" % rid)
    # the same requests replayed by msrep_serve give the same bits
    trace = [synth.Request(rid, 0.0, k, steps) for rid, k, steps in reqs[:6]]
    res, _ = serving.serve(pool, trace, budget_bytes=2 << 30, vtype=vt, seed=SEED, keep_y=True)
    for (rid, _, _), r in zip(reqs[:6], res):
        assert np.array_equal(r.y, ys[rid]), rid


def test_incremental_server_busy_and_budget():
    """A full queue refuses submissions with MSREP_ERR_BUSY; a request whose
    matrix can never fit the arena completes with MSREP_ERR_BUDGET while the
    others finish."""
    pool = _pool(4, m_hi=20_000)
    big = max(range(len(pool)), key=lambda k: pool[k].nnz)
    small = min(range(len(pool)), key=lambda k: pool[k].nnz)
    # one slot: a long request holds it while others wait in a queue of 2
    with serving.Server(pool, 2 << 30, max_slots=1, seed=SEED, max_queue=2) as S:
        S.submit(0, big, 3000)
        busy = 0
        for rid in range(1, 8):
            try:
                S.submit(rid, small, 2)
            except pk.MsrepError as e:
                assert e.status == -6
                busy += 1
        assert busy > 0
        st = S.close()
    assert st["n_done"] == 8 - busy
    # a budget too small for the largest matrix
    A = pool[big]
    budget = 4 * (A.m + A.nnz) + 8 * A.nnz // 2
    with serving.Server(pool, budget, seed=SEED) as S:
        S.submit(100, big, 2)
        S.submit(101, small, 2, keep_y=True)
        out = {}
        for _ in range(400):
            for c in S.poll(timeout_ms=50):
                out[c.rid] = c.status
            if len(out) == 2:
                break
        assert out == {100: -5, 101: 0}, out
        ref, s = _oracle_y(pool[small], 101, 2, pk.F64)
        assert_close(S.y_of(101), ref, s, F64_TOL, "small request beside a refused one")
