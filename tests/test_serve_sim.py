"""CPU tests of the serving scheduler through msrep_serve_simulate (the same
admission / residency / continuous-batching code as msrep_serve, driven by a
virtual device clock)."""
import os

import numpy as np
import pytest

import synth

pk = pytest.importorskip("paper_2209_07552_amd")
from paper_2209_07552_amd import serving  # noqa: E402

if not os.path.exists(pk.lib_path()):
    pytest.skip("libmsrep.so not built", allow_module_level=True)


def _pool(count=6, m_hi=20_000):
    return [A for A, _ in synth.batched_set(count, seed=3, m_lo=500, m_hi=m_hi)]


SPT = 64  # the library's default steps per tick: a request's X and Y have min(steps, SPT) columns


def _bytes(A, np_, xb=8, steps=1):
    r = lambda b: (b + 255) // 256 * 256
    c = max(1, min(steps, SPT))
    ld = min(8, c)
    cb = ld * (-(-c // ld))  # whole blocks of ld columns
    # a resident matrix holds its arrays and its partitions (shared by every
    # request on it); a request holds its vectors and carries
    mat = r(4 * (A.m + 1)) + r(4 * A.nnz) + r(xb * A.nnz) + r(40 * np_) + r(4 * (A.m + 2 * np_))
    req = r(cb * xb * A.n) + r(cb * xb * A.m) + r(16 * np_ * c)
    return mat, req


def _np(A):
    return max(1, -(-A.nnz // 1024))


def test_all_complete_with_a_large_budget():
    pool = _pool()
    trace = synth.serving_trace(40, rate=20000.0, pool=len(pool), seed=1, k_lo=3, k_hi=12)
    res, st = serving.serve(pool, trace, budget_bytes=1 << 34, simulate=True)
    assert all(r.status == 0 for r in res)
    for r, q in zip(res, trace):
        assert r.t_arrive == q.t_arrive and r.t_admit >= r.t_arrive and r.t_done > r.t_admit
    assert st["n_done"] == 40 and st["n_failed"] == 0
    assert st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    # continuous batching: far fewer ticks than SpMV steps
    assert st["ticks"] < sum(q.steps for q in trace)
    assert st["peak_active"] > 1


def test_request_that_can_never_fit_fails_alone():
    pool = _pool()
    big = max(range(len(pool)), key=lambda k: pool[k].nnz)
    mat, req = _bytes(pool[big], _np(pool[big]), steps=5)
    budget = mat + req - 4096  # too small for the largest matrix only
    others = [k for k in range(len(pool))
              if sum(_bytes(pool[k], _np(pool[k]), steps=4)) + 512 <= budget]
    trace = [synth.Request(0, 0.0, big, 5)] + [synth.Request(i + 1, 1e-4 * i, k, 4)
                                               for i, k in enumerate(others)]
    res, st = serving.serve(pool, trace, budget_bytes=budget, simulate=True)
    assert res[0].status == pk._abi.MsrepError(-5, "").status
    assert all(r.status == 0 for r in res[1:])
    assert st["peak_bytes"] <= budget


def test_budget_bounds_residency_and_queues():
    pool = _pool()
    # room for one request of any matrix (at the most steps) at a time
    budget = max(sum(_bytes(A, _np(A), steps=6)) for A in pool) + 1024
    trace = synth.serving_trace(30, rate=1e6, pool=len(pool), seed=2, k_lo=2, k_hi=6)
    res, st = serving.serve(pool, trace, budget_bytes=budget, simulate=True)
    assert all(r.status == 0 for r in res)
    assert st["peak_bytes"] <= budget
    # requests on different matrices that cannot both fit never overlapped
    size = [sum(_bytes(pool[q.matrix], _np(pool[q.matrix]), steps=q.steps)) for q in trace]
    iv = sorted((r.t_admit, r.t_done, q.matrix, size[i])
                for i, (r, q) in enumerate(zip(res, trace)))
    for (a0, d0, m0, s0), (a1, d1, m1, s1) in zip(iv, iv[1:]):
        if m0 != m1 and s0 + s1 > budget:
            assert a1 >= d0 - 1e-12


def test_steps_per_tick_batches_a_requests_steps():
    """A tick runs up to steps_per_tick steps of each request: one step per
    tick needs at least as many ticks as the longest request has steps;
    eight per tick need far fewer, and every request still completes."""
    pool = _pool()
    trace = synth.serving_trace(20, rate=200.0, pool=len(pool), seed=6, k_lo=10, k_hi=40)
    one = serving.serve(pool, trace, budget_bytes=1 << 34, simulate=True, steps_per_tick=1)
    eight = serving.serve(pool, trace, budget_bytes=1 << 34, simulate=True, steps_per_tick=8)
    assert all(r.status == 0 for r in one[0]) and all(r.status == 0 for r in eight[0])
    assert one[1]["ticks"] >= max(q.steps for q in trace)
    assert eight[1]["ticks"] * 4 <= one[1]["ticks"]
    assert eight[1]["p50_ms"] < one[1]["p50_ms"]
    # a tick never holds more than 240 requests: 300 requests of 64 steps
    # arriving at once (eight ticks' worth each) fill ticks to 240 and take
    # at least 300*8/240 ticks
    burst = [synth.Request(i, 0.0, i % len(pool), 64) for i in range(300)]
    res, st = serving.serve(pool, burst, budget_bytes=1 << 36, max_slots=300, simulate=True,
                            steps_per_tick=8)
    assert all(r.status == 0 for r in res)
    assert st["peak_active"] == 240 and st["ticks"] >= 300 * 8 // 240


def test_max_slots_one_serialises():
    pool = _pool()
    trace = synth.serving_trace(12, rate=1e6, pool=len(pool), seed=4, k_lo=2, k_hi=5)
    res, st = serving.serve(pool, trace, budget_bytes=1 << 34, max_slots=1, simulate=True)
    iv = sorted((r.t_admit, r.t_done) for r in res)
    for (a0, d0), (a1, d1) in zip(iv, iv[1:]):
        assert a1 >= d0 - 1e-12
    assert st["peak_active"] == 1


def test_simulation_is_deterministic():
    pool = _pool()
    trace = synth.serving_trace(25, rate=5000.0, pool=len(pool), seed=5, k_lo=3, k_hi=9)
    a = serving.serve(pool, trace, budget_bytes=1 << 30, simulate=True)
    b = serving.serve(pool, trace, budget_bytes=1 << 30, simulate=True)
    assert [(r.t_admit, r.t_done) for r in a[0]] == [(r.t_admit, r.t_done) for r in b[0]]
    assert a[1] == b[1]


def test_bad_requests_rejected():
    pool = _pool(2)
    with pytest.raises(pk.MsrepError):
        serving.serve(pool, [synth.Request(0, 0.0, 5, 3)], budget_bytes=1 << 30, simulate=True)
    with pytest.raises(pk.MsrepError):
        serving.serve(pool, [synth.Request(0, 0.0, 0, 0)], budget_bytes=1 << 30, simulate=True)


def test_x_generator_matches_published_definition():
    xs = [serving.x_value(11, 7, 3, c) for c in range(16)]
    assert np.array_equal(np.array(xs), synth.serving_x(16, 11, 7, 3))
    # known SplitMix64 output for key 0 (first output of a generator seeded 0)
    assert int(synth.splitmix64(np.array([0], np.uint64))[0]) == 0xE220A8397B1DCDAF


def test_tick_cap_follows_load():
    """How many steps of a request a tick runs follows the load: a lone
    request runs all its steps in one tick; 240 requests at once, whose
    64-step ticks would hold far more (partition, pass) items than the GPU
    has resident wavefronts, run 8 steps each per tick."""
    pool = _pool()
    nps = [64] * len(pool)
    lone, st = serving.serve(pool, [synth.Request(0, 0.0, 0, 40)], budget_bytes=1 << 34,
                             simulate=True, nps=nps)
    assert lone[0].status == 0 and st["ticks"] == 1
    burst = [synth.Request(i, 0.0, i % len(pool), 64) for i in range(240)]
    res, st = serving.serve(pool, burst, budget_bytes=1 << 36, max_slots=240, simulate=True,
                            nps=nps)
    assert all(r.status == 0 for r in res)
    assert st["ticks"] >= 8  # 8 steps of each request per tick, once all are in


def test_large_requests_reserve_eight_columns():
    """A request reserves min(steps, steps_per_tick) columns of X and Y,
    except when those would take more than a sixteenth of the arena: then 8
    (what a tick under load runs), so that a small arena holds more
    requests."""
    pool = _pool()
    A = pool[0]
    mat, full = _bytes(A, _np(A), steps=40)
    _, eight = _bytes(A, _np(A), steps=8)
    assert eight < full
    for budget, want in ((16 * full + (1 << 20), full), (16 * full - 256, eight)):
        res, st = serving.serve(pool, [synth.Request(0, 0.0, 0, 40)], budget_bytes=budget,
                                simulate=True)
        assert res[0].status == 0
        assert st["peak_bytes"] == mat + want, (budget, st["peak_bytes"], mat + want)


def test_requests_on_one_matrix_share_its_partitions():
    """A resident matrix holds its partitions once: two requests on it,
    admitted together, take the matrix's bytes (arrays and partitions) once
    and their own vectors and carries each."""
    pool = _pool()
    A = pool[2]
    mat, req = _bytes(A, _np(A), steps=5)
    trace = [synth.Request(0, 0.0, 2, 5), synth.Request(1, 0.0, 2, 5)]
    res, st = serving.serve(pool, trace, budget_bytes=1 << 34, simulate=True)
    assert all(r.status == 0 for r in res)
    assert st["peak_bytes"] == mat + 2 * req
