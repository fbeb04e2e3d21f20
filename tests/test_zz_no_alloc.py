"""msrep_spmv_noalloc (boundary carries in the library's static device
scratch) against msrep_spmv with a workspace, on two calls in a row, the
second with a smaller matrix, and against the oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import F64_TOL, F32_TOL, assert_close, device_mat, oracle_y, stored_values

pytestmark = pytest.mark.gpu


def _run(A, fmt, vt, np_, tune, alpha=1.0, beta=0.0, seed=3):
    import torch
    import paper_2209_07552_amd as pk
    print("noalloc case: fmt=%s vt=%d m=%d nnz=%d np=%d tune=%s beta=%g"
          % (fmt, vt, A.m, A.ptr[-1], np_, tune, beta), flush=True)
    dev = torch.device("cuda:0")
    M, v64 = device_mat(A, fmt, vt)
    P = pk.msrep_build_partition(M, np_)
    x64 = np.random.default_rng(seed).uniform(-1, 1, A.n)
    y0 = np.random.default_rng(seed + 1).uniform(-1, 1, A.m)
    xs, xo = stored_values(x64, pk.F64 if vt == pk.F64 else pk.F32)
    vdt = torch.float64 if vt == pk.F64 else torch.float32
    x = torch.from_numpy(np.asarray(xs)).to(dev, vdt)
    ya = torch.from_numpy(y0).to(dev, vdt)
    yb = ya.clone()
    pk.msrep_spmv(M, P, x, ya, alpha, beta, tune=tune)
    pk.msrep_spmv_noalloc(M, P, x, yb, alpha, beta, tune=tune)
    torch.cuda.synchronize()
    a, b = ya.cpu().numpy(), yb.cpu().numpy()
    # same kernels, same launch shape: bit-identical
    assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), "noalloc differs from msrep_spmv"
    yin = np.asarray(y0.astype(np.float32), np.float64) if vt != pk.F64 else y0
    ref, s = oracle_y(A, fmt, v64, xo if vt != pk.F64 else x64, alpha, beta, yin)
    assert_close(b, ref, s, F64_TOL if vt == pk.F64 else F32_TOL, "noalloc %s" % fmt)


@pytest.mark.parametrize("fmt", ["csr", "coo"])
def test_noalloc_two_calls_second_smaller(fmt):
    import paper_2209_07552_amd as pk
    big, _ = synth.rmat_csr(scale=14, edge_factor=8, seed=5)
    small, _ = synth.rmat_csr(scale=10, edge_factor=4, seed=6)
    t = pk.Tune(k_per_lane=4, waves_per_wg=4, resident=1)
    _run(big, fmt, pk.F64, 997, t)
    _run(small, fmt, pk.F64, 61, None, alpha=-0.5, beta=0.25)


def test_noalloc_low_precision_and_stencil():
    import paper_2209_07552_amd as pk
    S, _ = synth.stencil7_csr(24)
    _run(S, "csr", pk.F32, 2000, None, beta=0.5)
    T, _ = synth.stencil7_csr(9)
    _run(T, "coo", pk.BF16, 33, None)


def test_noalloc_limits():
    import torch
    import paper_2209_07552_amd as pk
    A, _ = synth.rmat_csr(scale=8, edge_factor=4, seed=1)
    M, _ = device_mat(A, "csc", pk.F64)
    P = pk.msrep_build_partition(M, 4)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    y = torch.zeros(A.m, dtype=torch.float64, device="cuda:0")
    with pytest.raises(pk.MsrepError) as e:
        pk.msrep_spmv_noalloc(M, P, x, y)
    assert e.value.status == -7
    assert pk.msrep_spmv_noalloc_max_parts() == 1 << 19
