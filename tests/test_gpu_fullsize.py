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
@pytest.mark.parametrize("fmt", ["csr", "csc", "coo"])
def test_full_size_bench_configuration(workload, fmt):
    import bench
    A, x, H = _workload(workload)
    npw, k, wpb, pf, res = bench.DEFAULT_TUNES[workload][fmt]
    np_ = -(-A.nnz // npw)
    a, b, v = H[fmt]
    kind = {"csr": pk.CSR, "csc": pk.CSC, "coo": pk.COO}[fmt]
    if fmt == "coo":
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
