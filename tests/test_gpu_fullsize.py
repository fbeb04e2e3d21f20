"""GPU parity at the benchmark's full sizes and launch configuration: R-MAT
scale 20 (16.09M nonzeros) and the 256^3 7-point stencil (117M nonzeros), in
every format, with the partition size and launch shape bench.py times and
through the entry point it times (msrep_spmv_prepare once, then
msrep_spmv_prepared), plus plain msrep_spmv.  The FP64 oracle computes every
output (it takes seconds at these sizes), so all m results are compared
element by element within 1e-12 of (|A||x|)_i."""
import numpy as np
import pytest

import synth
from gpu_common import F64_TOL, assert_close, host_formats, oracle_y

torch = pytest.importorskip("torch")
pk = pytest.importorskip("paper_2209_07552_amd")

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

_cache = {}


def _workload(name):
    """(A, x, host formats) of the benchmark workload, generated once."""
    if name not in _cache:
        if name == "rmat20":
            A, x = synth.rmat_csr(scale=20, edge_factor=16, seed=0)
        else:
            A, x = synth.stencil7_csr(256, seed=0)
        _cache[name] = (A, x, host_formats(A))
    return _cache[name]


@pytest.mark.parametrize("workload", ["rmat20", "stencil256"])
@pytest.mark.parametrize("fmt", ["csr", "csc", "coo", "coo_col"])
def test_full_size_bench_configuration(workload, fmt):
    import bench
    A, x, H = _workload(workload)
    npw, k, wpb, pf, res = bench.DEFAULT_TUNES[workload][fmt]
    np_ = -(-A.nnz // npw)
    a, b, v = H[fmt]
    kind = {"csr": pk.CSR, "csc": pk.CSC, "coo": pk.COO, "coo_col": pk.COO_COL}[fmt]
    if fmt in ("coo", "coo_col"):
        M = pk.Mat(kind, pk.F64, A.m, A.n, idx=a, idx2=b, val=v)
    else:
        M = pk.Mat(kind, pk.F64, A.m, A.n, ptr=a, idx=b, val=v)
    dev = torch.device("cuda:0")
    P = pk.msrep_build_partition(M, np_)
    tune = pk.Tune(k_per_lane=k, waves_per_wg=wpb, pipeline=pf, resident=res)
    xd = torch.from_numpy(x).to(dev)
    ws = pk.msrep_spmv_prepare(M, P)
    y1 = torch.full((A.m,), float("nan"), dtype=torch.float64, device=dev)
    pk.msrep_spmv_prepared(M, P, xd, y1, ws, 1.0, 0.0, tune)
    y2 = torch.full((A.m,), float("nan"), dtype=torch.float64, device=dev)
    pk.msrep_spmv(M, P, xd, y2, 1.0, 0.0, tune)
    torch.cuda.synchronize()
    ref, s = oracle_y(A, fmt, v, x)
    what = "%s %s np%d" % (workload, fmt, np_)
    assert_close(y1.cpu().numpy(), ref, s, F64_TOL, what + " prepared")
    assert_close(y2.cpu().numpy(), ref, s, F64_TOL, what)
    del M, P, ws, xd, y1, y2
    torch.cuda.empty_cache()


def _mat(A, H, fmt, vt, val=None):
    from gpu_common import stored_values
    a, b, v = H[fmt]
    if val is not None:
        v = val
    sv, v64 = stored_values(v, vt)
    kind = {"csr": pk.CSR, "csc": pk.CSC, "coo": pk.COO, "coo_col": pk.COO_COL}[fmt]
    if fmt in ("coo", "coo_col"):
        return pk.Mat(kind, vt, A.m, A.n, idx=a, idx2=b, val=sv), v64
    return pk.Mat(kind, vt, A.m, A.n, ptr=a, idx=b, val=sv), v64


def _spmv_bench_config(workload, fmt, M, nnz, x, vt):
    import bench
    npw, k, wpb, pf, res = bench.DEFAULT_TUNES[workload][fmt]
    P = pk.msrep_build_partition(M, -(-nnz // npw))
    tune = pk.Tune(k_per_lane=k, waves_per_wg=wpb, pipeline=pf, resident=res)
    dev = torch.device("cuda:0")
    xd = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    ws = pk.msrep_spmv_prepare(M, P)
    y = torch.full((M.m,), float("nan"), dtype=xd.dtype, device=dev)
    pk.msrep_spmv_prepared(M, P, xd, y, ws, 1.0, 0.0, tune)
    torch.cuda.synchronize()
    out = y.cpu().numpy().astype(np.float64)
    del P, ws, xd, y
    return out


@pytest.mark.parametrize("vt", [0, 1, 2])
@pytest.mark.parametrize("fmt", ["csr", "csc", "coo", "coo_col"])
def test_full_size_stencil_times_ones_exact(fmt, vt):
    """256^3 stencil times ones: y_i = 6 - (in-grid neighbours of i), a small
    integer, exact in every value type at the full 16.7M rows."""
    A, _, H = _workload("stencil256")
    M, _ = _mat(A, H, fmt, vt)
    xdt = np.float64 if vt == 0 else np.float32
    y = _spmv_bench_config("stencil256", fmt, M, A.nnz, np.ones(A.n, xdt), vt)
    g = 256
    r = np.arange(A.m)
    want = np.zeros(A.m)
    for c in (r % g, (r // g) % g, r // (g * g)):
        want += (c == 0).astype(np.float64) + (c == g - 1).astype(np.float64)
    assert np.array_equal(y, want), (fmt, vt)
    del M
    torch.cuda.empty_cache()


@pytest.mark.parametrize("workload", ["rmat20", "stencil256"])
@pytest.mark.parametrize("fmt", ["csr", "csc", "coo", "coo_col"])
def test_full_size_dyadic_bit_exact(workload, fmt):
    """Dyadic values and x (k/256, |k| <= 256): every partial sum is exact in
    FP64, so the full-size result must equal the oracle's bit for bit, which
    pins the partition split and the boundary merge at the benchmark's
    configuration."""
    A, _, H = _workload(workload)
    rng = np.random.default_rng(31)
    x = synth.dyadic(rng, A.n)
    val = None
    if workload == "rmat20":  # the stencil's 6 and -1 are dyadic already
        v_csr = synth.dyadic(rng, A.nnz)
        val = v_csr
        if fmt in ("csc", "coo_col"):
            import oracle
            _, _, _, p = oracle.transpose(A.m, A.n, A.ptr, A.col)
            val = v_csr[p]
    M, v64 = _mat(A, H, fmt, pk.F64, val)
    y = _spmv_bench_config(workload, fmt, M, A.nnz, x, pk.F64)
    ref, _ = oracle_y(A, fmt, v64, x)
    assert np.array_equal(y, ref), (workload, fmt, int(np.sum(y != ref)))
    del M
    torch.cuda.empty_cache()


@pytest.mark.parametrize("vt", [1, 2])
@pytest.mark.parametrize("workload", ["rmat20", "stencil256"])
@pytest.mark.parametrize("fmt", ["csr", "csc", "coo", "coo_col"])
def test_full_size_low_precision_random_x(workload, fmt, vt):
    """FP32 and BF16 stored values with the benchmark's random x (rounded to
    FP32), at full size and in the benchmark's configuration: every row
    within 1e-5 of (|A||x|)_i against the FP64 oracle on the stored values."""
    from gpu_common import F32_TOL
    A, x, H = _workload(workload)
    M, v64 = _mat(A, H, fmt, vt)
    x32 = x.astype(np.float32)
    y = _spmv_bench_config(workload, fmt, M, A.nnz, x32, vt)
    ref, s = oracle_y(A, fmt, v64, x32.astype(np.float64))
    assert_close(y, ref, s, F32_TOL, "%s %s vt%d" % (workload, fmt, vt))
    del M
    torch.cuda.empty_cache()
