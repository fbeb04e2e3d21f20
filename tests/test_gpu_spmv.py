"""GPU parity: partition metadata bit-exact against the oracle, SpMV within
the stated tolerances (FP64 1e-12, FP32 1e-5 of |alpha||A||x| + |beta||y|),
exact on dyadic inputs and on the stencil times ones, deterministic for the
row-split formats.  Every call goes through the C ABI."""
import numpy as np
import pytest

import oracle
import synth
from conftest import load_golden
from gpu_common import F32_TOL, F64_TOL, assert_close, device_mat, host_formats, oracle_y

torch = pytest.importorskip("torch")
pk = pytest.importorskip("paper_2209_07552_amd")

pytestmark = pytest.mark.gpu

FMTS = ["csr", "csc", "coo", "coo_col"]
BUCKETED = ("csc", "coo_col")  # the column-merge path: its tune picks the product layout


def _dev():
    return torch.device("cuda:0")


def _golden_csr():
    kv, _ = load_golden("example_6x6.txt")
    m, n = int(kv["m"][0]), int(kv["n"][0])
    A = synth.Csr(m, n, np.array(kv["row_ptr"], np.int32), np.array(kv["col_idx"], np.int32),
                  np.array(kv["val"], np.float64), name="golden")
    return A, np.array(kv["x"], np.float64)


def _tiny_set():
    """Adversarial small matrices: empty, all-empty rows, one dense row, long
    rows crossing many partitions and chunks, leading/trailing empty rows."""
    out = [_golden_csr()]
    rng = np.random.default_rng(5)

    def mk(counts, n, name):
        counts = np.asarray(counts, np.int64)
        rows = np.repeat(np.arange(len(counts)), counts)
        cols = np.concatenate([np.sort(rng.choice(n, c, replace=False)) for c in counts]) \
            if counts.sum() else np.zeros(0, np.int64)
        ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
        A = synth.Csr(len(counts), n, ptr, cols.astype(np.int32), rng.uniform(-1, 1, len(rows)),
                      name=name)
        return A, rng.uniform(-1, 1, n)

    out.append(mk([0, 0, 0], 5, "all-empty"))
    out.append(mk([7], 9, "one-row"))
    out.append(mk([0, 0, 3000, 0, 1, 0, 0], 4000, "long-row"))
    out.append(mk([0] * 50 + [2] * 10 + [0] * 40, 64, "lead-trail-empty"))
    out.append(mk(rng.integers(0, 40, 300) * (rng.random(300) < 0.5), 200, "ragged"))
    out.append(mk([5000, 1, 2000, 0, 3], 6000, "two-long"))
    return out


# --------------------------------------------------------------- partitions
def _part_compare(A, fmt, np_, split="nnz"):
    M, _ = device_mat(A, fmt, pk.F64)
    P = pk.msrep_build_partition(M, np_, split=pk.SPLIT_ROWS if split == "rows" else pk.SPLIT_NNZ)
    torch.cuda.synchronize()
    rec, lp = P.host()
    H = host_formats(A)
    if fmt == "coo":
        R = oracle.partition_coo(A.m, H["coo"][0], np_, split)
    elif fmt == "coo_col":
        R = oracle.partition_coo_col(A.n, H["coo_col"][1], np_, split)
    else:
        rows = A.m if fmt == "csr" else A.n
        R = oracle.partition_ptr(rows, H[fmt][0], np_, split)
    for f in ("start_idx", "end_idx", "start_row", "end_row", "start_flag", "end_flag",
              "lptr_off"):
        assert np.array_equal(rec[f], getattr(R, f)), (A.name, fmt, np_, f)
    if fmt in ("csr", "csc"):
        for i in range(np_):
            o = int(R.lptr_off[i])
            k = int(R.end_row[i] - R.start_row[i] + 2)
            assert np.array_equal(lp[o:o + k], R.lptr[o:o + k]), (A.name, fmt, np_, i)
        assert int(P.lptr_len.item()) == R.lptr_len


@pytest.mark.parametrize("fmt", FMTS)
def test_partition_tiny_all_np(fmt):
    for A, _ in _tiny_set():
        for np_ in sorted({1, 2, 3, 4, 7, 12, A.nnz + 1, A.nnz + 2, 64}):
            _part_compare(A, fmt, np_)


@pytest.mark.parametrize("fmt", FMTS)
def test_partition_uniform_and_rmat(fmt):
    A, _ = synth.uniform_csr(4096, 4096, 16, seed=0)
    for np_ in (8, 7, 3, 256):
        _part_compare(A, fmt, np_)
    B, _ = synth.rmat_csr(scale=14, edge_factor=16, seed=0)
    for np_ in (1, 37, 256, 4096, 100_000):
        _part_compare(B, fmt, np_)


def test_partition_uniform_np8_no_partial_rows():
    A, _ = synth.uniform_csr(4096, 4096, 16, seed=0)
    M, _ = device_mat(A, "csr", pk.F64)
    rec, _ = pk.msrep_build_partition(M, 8).host()
    assert np.all(rec["start_flag"] == 0) and np.all(rec["end_flag"] == 0)
    assert np.all(rec["end_idx"] - rec["start_idx"] + 1 == 8192)


# --------------------------------------------------------------------- SpMV
def _run(A, x64, fmt, vt, np_, alpha=1.0, beta=0.0, y_in=None, tune=None, M=None, v64=None):
    if M is None:
        M, v64 = device_mat(A, fmt, vt)
    P = pk.msrep_build_partition(M, np_)
    vdt = torch.float64 if vt == pk.F64 else torch.float32
    xs = np.asarray(x64, np.float64 if vt == pk.F64 else np.float32)
    x = torch.from_numpy(np.ascontiguousarray(xs)).to(_dev())
    if beta == 0.0:
        y = torch.full((A.m,), float("nan"), dtype=vdt, device=_dev())  # must not be read
    else:
        y = torch.from_numpy(np.asarray(y_in, xs.dtype)).to(_dev())
    pk.msrep_spmv(M, P, x, y, alpha, beta, tune)
    torch.cuda.synchronize()
    x_used = xs.astype(np.float64)
    yi = None if beta == 0.0 else np.asarray(y_in, xs.dtype).astype(np.float64)
    ref, scale = oracle_y(A, fmt, v64, x_used, alpha, beta, yi)
    return y.cpu().numpy().astype(np.float64), ref, scale


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("vt", [0, 1, 2])
def test_spmv_tiny_set(fmt, vt):
    tol = F64_TOL if vt == 0 else F32_TOL
    rng = np.random.default_rng(1)
    for A, x in _tiny_set():
        for np_ in sorted({1, 2, 3, 7, A.nnz + 2, 40}):
            for alpha, beta in ((1.0, 0.0), (-0.5, 2.0)):
                y_in = rng.uniform(-1, 1, A.m)
                y, ref, s = _run(A, x, fmt, vt, np_, alpha, beta, y_in)
                assert_close(y, ref, s, tol, "%s %s vt%d np%d a%g b%g" % (A.name, fmt, vt, np_,
                                                                         alpha, beta))


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("tune", [(4, 4, 0), (8, 4, 0), (4, 1, 1), (8, 8, 1)])
def test_spmv_uniform_4096(fmt, tune):
    A, x = synth.uniform_csr(4096, 4096, 16, seed=0)
    t = pk.Tune(k_per_lane=tune[0], waves_per_wg=tune[1], resident=tune[2])
    for np_ in (8, 7, 3, 1024):
        y, ref, s = _run(A, x, fmt, pk.F64, np_, tune=t)
        assert_close(y, ref, s, F64_TOL, "uniform %s np%d" % (fmt, np_))


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("vt", [0, 1, 2])
def test_spmv_rmat14(fmt, vt):
    A, x = synth.rmat_csr(scale=14, edge_factor=16, seed=3)
    tol = F64_TOL if vt == 0 else F32_TOL
    rng = np.random.default_rng(2)
    y_in = rng.uniform(-1, 1, A.m)
    M, v64 = device_mat(A, fmt, vt)
    for np_ in (1, 37, 256, 2048):
        for k, res in ((4, 0), (8, 0), (4, 1)):
            y, ref, s = _run(A, x, fmt, vt, np_, 1.25, 0.5, y_in,
                             tune=pk.Tune(k_per_lane=k, resident=res), M=M, v64=v64)
            assert_close(y, ref, s, tol, "rmat14 %s vt%d np%d k%d res%d" % (fmt, vt, np_, k, res))


@pytest.mark.parametrize("fmt", FMTS)
def test_dyadic_bit_exact_any_np(fmt):
    """Dyadic values and x make every partial sum exact: the result must be
    bit-identical to the oracle for every np, which pins the merge."""
    A, _ = synth.rmat_csr(scale=15, edge_factor=16, seed=4)
    rng = np.random.default_rng(4)
    A.val = synth.dyadic(rng, A.nnz)
    x = synth.dyadic(rng, A.n)
    M, v64 = device_mat(A, fmt, pk.F64)
    for np_ in (1, 5, 256, 4096, A.nnz + 7):
        for res in (0, 1, 2):  # column merge: the two product layouts and the row windows
            if res == 2 and fmt not in BUCKETED:
                continue
            t = pk.Tune(pipeline=1 + res) if fmt in BUCKETED else pk.Tune(resident=res)
            y, ref, _ = _run(A, x, fmt, pk.F64, np_, M=M, v64=v64, tune=t)
            assert np.array_equal(y, ref), (fmt, np_, res)


def test_stencil_times_ones_exact():
    A, _ = synth.stencil7_csr(64)
    r = np.arange(A.m)
    g = 64
    i, j, k = r % g, (r // g) % g, r // (g * g)
    want = sum(((c == 0).astype(int) + (c == g - 1).astype(int)) for c in (i, j, k)).astype(float)
    for fmt in FMTS:
        for vt in (0, 1, 2):
            y, _, _ = _run(A, np.ones(A.n), fmt, vt, 1000)
            assert np.array_equal(y, want), (fmt, vt)


@pytest.mark.parametrize("fmt", ["csr", "coo"])
@pytest.mark.parametrize("vt", [0, 1])
def test_merge_rows_spanning_many_blocks(fmt, vt):
    """Rows split over thousands of partitions: the boundary merge must carry
    a row's sum across many blocks of partitions and across empty ones."""
    rng = np.random.default_rng(8)
    counts = np.array([0, 40000, 3, 0, 9000, 1, 0, 70000, 2, 5], np.int64)
    n = 80000
    cols = np.concatenate([np.sort(rng.choice(n, c, replace=False)) for c in counts])
    ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    A = synth.Csr(len(counts), n, ptr, cols.astype(np.int32), rng.uniform(-1, 1, cols.size),
                  name="many-blocks")
    x = rng.uniform(-1, 1, n)
    y_in = rng.uniform(-1, 1, A.m)
    tol = F64_TOL if vt == 0 else F32_TOL
    M, v64 = device_mat(A, fmt, vt)
    for np_ in (A.nnz // 3, A.nnz // 64, 1000, A.nnz + 300):
        y, ref, s = _run(A, x, fmt, vt, np_, -1.5, -0.75, y_in, M=M, v64=v64)
        assert_close(y, ref, s, tol, "many-blocks %s vt%d np%d" % (fmt, vt, np_))


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("vt", [0, 1])
def test_runs_of_empty_rows_and_columns(fmt, vt):
    """Nonzeros separated by thousands of empty rows and columns: one chunk
    of a partition spans many rounds of pointer words, and the rows between
    its nonzeros must still get beta*y."""
    rng = np.random.default_rng(9)
    m = n = 300_000
    rows = np.sort(rng.choice(m, 700, replace=False))
    rows = np.concatenate([rows, np.full(40, rows[350])])  # one row with 41 entries
    cols = rng.choice(n, rows.size, replace=True)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    keep = np.ones(rows.size, bool)
    keep[1:] = (rows[1:] != rows[:-1]) | (cols[1:] != cols[:-1])
    rows, cols = rows[keep], cols[keep]
    ptr = np.zeros(m + 1, np.int64)
    np.add.at(ptr, rows + 1, 1)
    ptr = np.cumsum(ptr).astype(np.int32)
    A = synth.Csr(m, n, ptr, cols.astype(np.int32), rng.uniform(-1, 1, rows.size), name="empty-runs")
    x = rng.uniform(-1, 1, n)
    y_in = rng.uniform(-1, 1, m)
    tol = F64_TOL if vt == 0 else F32_TOL
    M, v64 = device_mat(A, fmt, vt)
    for np_ in (1, 3, 64, A.nnz + 5):
        for beta in (0.0, 0.5):
            y, ref, s = _run(A, x, fmt, vt, np_, 2.0, beta, y_in, M=M, v64=v64)
            assert_close(y, ref, s, tol, "empty-runs %s vt%d np%d b%g" % (fmt, vt, np_, beta))


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("vt", [0, 1])
def test_prepared_spmv_repeats_with_fresh_x(fmt, vt):
    """msrep_spmv_prepare once, then msrep_spmv_prepared with fresh x, alpha
    and beta (CSC in both product layouts), with plain msrep_spmv calls on
    another matrix in between: every result matches the oracle."""
    A, _ = synth.rmat_csr(scale=14, edge_factor=16, seed=12)
    B, xb = synth.uniform_csr(3000, 3000, 9, seed=2)
    tol = F64_TOL if vt == 0 else F32_TOL
    xdt = np.float64 if vt == 0 else np.float32
    tdt = torch.float64 if vt == 0 else torch.float32
    M, v64 = device_mat(A, fmt, vt)
    MB, _ = device_mat(B, fmt, vt)
    rng = np.random.default_rng(21)
    for np_ in (7, 2048):
        P = pk.msrep_build_partition(M, np_)
        PB = pk.msrep_build_partition(MB, 33)
        ws = pk.msrep_spmv_prepare(M, P)
        for it in range(6):
            x = rng.uniform(-1, 1, A.n).astype(xdt)
            y_in = rng.uniform(-1, 1, A.m).astype(xdt)
            alpha, beta = (1.0, 0.0) if it % 2 == 0 else (-2.0, 0.25)
            xd = torch.from_numpy(x).to(_dev())
            yd = torch.from_numpy(y_in.copy()).to(_dev())
            tune = pk.Tune(pipeline=1 + it % 3) if fmt in BUCKETED else None
            pk.msrep_spmv_prepared(M, P, xd, yd, ws, alpha, beta, tune)
            # an unprepared SpMV of another matrix on the shared workspace
            yb = torch.zeros(B.m, dtype=tdt, device=_dev())
            pk.msrep_spmv(MB, PB, torch.from_numpy(xb.astype(xdt)).to(_dev()), yb)
            torch.cuda.synchronize()
            yi = None if beta == 0.0 else y_in.astype(np.float64)
            ref, sc = oracle_y(A, fmt, v64, x.astype(np.float64), alpha, beta, yi)
            assert_close(yd.cpu().numpy().astype(np.float64), ref, sc, tol,
                          "prepared %s vt%d np%d it%d" % (fmt, vt, np_, it))


@pytest.mark.parametrize("fmt", FMTS)
def test_equal_rows_baseline_partitions(fmt):
    """The paper's Baseline split (msrep_build_partition_rows: equal row or
    column blocks, unequal nonzeros, no split rows) is bit-exact against the
    oracle's, and the SpMV kernels take its records like equal-nnz ones."""
    rng = np.random.default_rng(17)
    for A, _ in _tiny_set():
        for np_ in sorted({1, 2, 3, 7, A.m + 2, 64}):
            _part_compare(A, fmt, np_, "rows")
    for A, x in (synth.rmat_csr(scale=14, edge_factor=16, seed=8), synth.stencil7_csr(48)):
        M, v64 = device_mat(A, fmt, pk.F64)
        y_in = rng.uniform(-1, 1, A.m)
        for np_ in (1, 7, 300):
            _part_compare(A, fmt, np_, "rows")
            P = pk.msrep_build_partition(M, np_, split=pk.SPLIT_ROWS)
            xd = torch.from_numpy(x).to(_dev())
            yd = torch.from_numpy(y_in.copy()).to(_dev())
            ws = pk.msrep_spmv_prepare(M, P)
            pk.msrep_spmv_prepared(M, P, xd, yd, ws, 1.5, -0.5)
            torch.cuda.synchronize()
            ref, sc = oracle_y(A, fmt, v64, x, 1.5, -0.5, y_in)
            assert_close(yd.cpu().numpy(), ref, sc, F64_TOL, "rows %s %s np%d" % (A.name, fmt, np_))


def _coo_any(A, vt, seed):
    """A as COO in a seeded random order: device Mat, and the shuffled host
    arrays with the FP64 image of the stored values."""
    from gpu_common import stored_values
    rows = oracle.csr_to_coo(A.m, A.ptr)
    perm = np.random.default_rng(seed).permutation(A.nnz)
    r, c, v = rows[perm], A.col[perm], A.val[perm]
    sv, v64 = stored_values(v, vt)
    M = pk.Mat(pk.COO_ANY, vt, A.m, A.n, idx=r, idx2=c, val=sv)
    return M, r, c, v64


@pytest.mark.parametrize("vt", [0, 1, 2])
def test_coo_any_order(vt):
    """COO in any order runs the bucketed (column-style merge) path: every
    result matches the oracle on the same shuffled arrays, for many np,
    both product layouts, alpha and beta; partitions are equal-nnz ranges."""
    tol = F64_TOL if vt == 0 else F32_TOL
    rng = np.random.default_rng(23)
    sets = _tiny_set()[1:] + [synth.rmat_csr(scale=14, edge_factor=16, seed=9),
                              synth.stencil7_csr(32)]
    for k, (A, x) in enumerate(sets):
        M, r, c, v64 = _coo_any(A, vt, 100 + k)
        xs = np.asarray(x, np.float64 if vt == pk.F64 else np.float32)
        xd = torch.from_numpy(np.ascontiguousarray(xs)).to(_dev())
        y_in = rng.uniform(-1, 1, A.m).astype(xs.dtype)
        for np_ in sorted({1, 7, 1000, A.nnz + 3}):
            P = pk.msrep_build_partition(M, np_)
            rec, _ = P.host()
            i = np.arange(np_, dtype=np.int64)
            assert np.array_equal(rec["start_idx"], i * A.nnz // np_)
            assert np.array_equal(rec["end_idx"], (i + 1) * A.nnz // np_ - 1)
            for pf in (1, 2, 3):
                for alpha, beta in ((1.0, 0.0), (-0.5, 2.0)):
                    y = torch.from_numpy(y_in.copy()).to(_dev())
                    pk.msrep_spmv(M, P, xd, y, alpha, beta, pk.Tune(pipeline=pf))
                    torch.cuda.synchronize()
                    yi = None if beta == 0.0 else y_in.astype(np.float64)
                    ref, sc = oracle.spmv_coo(A.m, A.n, r, c, v64, xs.astype(np.float64), alpha,
                                              beta, yi)
                    assert_close(y.cpu().numpy(), ref, sc, tol,
                                 "%s coo_any vt%d np%d pf%d b%g" % (A.name, vt, np_, pf, beta))


def test_coo_any_dyadic_bit_exact_and_prepared():
    """Dyadic inputs: bit-exact against the oracle for every np, also through
    msrep_spmv_prepare / msrep_spmv_prepared."""
    A, _ = synth.rmat_csr(scale=15, edge_factor=16, seed=4)
    rng = np.random.default_rng(4)
    A.val = synth.dyadic(rng, A.nnz)
    x = synth.dyadic(rng, A.n)
    M, r, c, v64 = _coo_any(A, pk.F64, 7)
    ref, _ = oracle.spmv_coo(A.m, A.n, r, c, v64, x)
    xd = torch.from_numpy(x).to(_dev())
    for np_ in (1, 5, 4096, A.nnz + 7):
        P = pk.msrep_build_partition(M, np_)
        y = torch.full((A.m,), float("nan"), dtype=torch.float64, device=_dev())
        pk.msrep_spmv(M, P, xd, y)
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), ref), np_
        ws = pk.msrep_spmv_prepare(M, P)
        for pf in (1, 2, 3):
            y2 = torch.full((A.m,), float("nan"), dtype=torch.float64, device=_dev())
            pk.msrep_spmv_prepared(M, P, xd, y2, ws, tune=pk.Tune(pipeline=pf))
            torch.cuda.synchronize()
            assert np.array_equal(y2.cpu().numpy(), ref), (np_, pf)


@pytest.mark.parametrize("fmt", ["csr", "coo"])
def test_deterministic(fmt):
    A, x = synth.rmat_csr(scale=14, edge_factor=16, seed=5)
    M, v64 = device_mat(A, fmt, pk.F64)
    y1, _, _ = _run(A, x, fmt, pk.F64, 777, M=M, v64=v64)
    y2, _, _ = _run(A, x, fmt, pk.F64, 777, M=M, v64=v64)
    assert np.array_equal(y1, y2)


def test_empty_shapes():
    for m, n in ((0, 0), (5, 0), (0, 5)):
        A = synth.Csr(m, n, np.zeros(m + 1, np.int32), np.zeros(0, np.int32), np.zeros(0))
        for fmt in FMTS:
            if m == 0:
                continue
            y, ref, s = _run(A, np.zeros(n), fmt, pk.F64, 3, 1.0, 3.0, np.arange(m, dtype=float))
            assert np.array_equal(y, ref)


def test_validate():
    A, _ = synth.rmat_csr(scale=10, edge_factor=8, seed=1)
    for fmt in FMTS:
        M, _ = device_mat(A, fmt, pk.F64)
        pk.msrep_validate(M)
    bad = A.col.copy()
    bad[17] = A.n + 3
    M = pk.Mat(pk.CSR, pk.F64, A.m, A.n, ptr=A.ptr, idx=bad, val=A.val)
    with pytest.raises(pk.MsrepError) as e:
        pk.msrep_validate(M)
    assert "position 17" in str(e.value)
    rows = oracle.csr_to_coo(A.m, A.ptr)
    rows[5], rows[6] = rows[6] + 1, rows[5]
    M = pk.Mat(pk.COO, pk.F64, A.m, A.n, idx=rows, idx2=A.col, val=A.val)
    with pytest.raises(pk.MsrepError):
        pk.msrep_validate(M)
    # column-sorted COO whose columns decrease at one position
    crow, ccol, cval = host_formats(A)["coo_col"]
    ccol = ccol.copy()
    ccol[40], ccol[41] = ccol[41] + 1, ccol[40]
    M = pk.Mat(pk.COO_COL, pk.F64, A.m, A.n, idx=crow, idx2=ccol, val=cval)
    with pytest.raises(pk.MsrepError) as e:
        pk.msrep_validate(M)
    assert "column indices are not sorted" in str(e.value)


def test_autotune_returns_a_valid_tune_and_correct_results():
    A, x = synth.rmat_csr(scale=14, edge_factor=16, seed=9)
    M, v64 = device_mat(A, "csr", pk.F64)
    xd = torch.from_numpy(x).to(_dev())
    t = pk.msrep_autotune(M, xd)
    assert t.k_per_lane in (4, 8) and t.waves_per_wg in (2, 4, 8) and t.resident in (0, 1)
    assert t.nnz_per_wave in (256, 512, 1024, 2048, 4096)
    np_ = max(1, -(-A.nnz // t.nnz_per_wave))
    y, ref, s = _run(A, x, "csr", pk.F64, np_, tune=t, M=M, v64=v64)
    assert_close(y, ref, s, F64_TOL, "autotuned")


@pytest.mark.parametrize("vt", [0, 1, 2])
def test_csc_many_buckets_and_pieces(vt):
    """CSC sums products by row bucket: R-MAT scale 16 puts a third of its
    nonzeros into the first bucket (several pieces merged in order) and the
    stencil spreads them over 64 buckets; both with beta != 0."""
    tol = F64_TOL if vt == 0 else F32_TOL
    rng = np.random.default_rng(11)
    for A, x in (synth.rmat_csr(scale=16, edge_factor=16, seed=6), synth.stencil7_csr(64)):
        M, v64 = device_mat(A, "csc", vt)
        y_in = rng.uniform(-1, 1, A.m)
        for np_ in (5, 4096, 100_000):
            for pf in (1, 2, 3):  # product records / value and row-offset arrays / row windows
                y, ref, s = _run(A, x, "csc", vt, np_, 0.75, -1.5, y_in, M=M, v64=v64,
                                 tune=pk.Tune(pipeline=pf))
                assert_close(y, ref, s, tol, "%s csc vt%d np%d pf%d" % (A.name, vt, np_, pf))


def test_kernel_timing_records_each_launch():
    """With timing on, every kernel of the call is bracketed by events: one
    CSR SpMV at np > 1 records the SpMV kernel and the boundary merge once
    each, the CSC path its five kernels and the scan; off records nothing."""
    A, x = synth.rmat_csr(scale=12, edge_factor=8, seed=2)
    pk.msrep_timing(True)
    try:
        _run(A, x, "csr", pk.F64, 64)
        t = pk.msrep_timing_read()
        assert set(t) == {"spmv_csr_seg", "merge_rows"}, t
        assert all(c == 1 and ms > 0 for c, ms in t.values()), t
        _run(A, x, "csc", pk.F64, 64)
        t = pk.msrep_timing_read()
        assert set(t) == {"csc_count", "csc_scan", "csc_scatter", "csc_plan", "csc_reduce",
                          "csc_merge"}, t
        pk.msrep_timing_only("csc_scatter")  # one kernel only
        _run(A, x, "csc", pk.F64, 64)
        t = pk.msrep_timing_read()
        assert set(t) == {"csc_scatter"} and t["csc_scatter"][0] == 1, t
        _run(A, x, "csr", pk.F64, 64)
        assert pk.msrep_timing_read() == {}
    finally:
        pk.msrep_timing_only(None)
        pk.msrep_timing(False)
    _run(A, x, "coo", pk.F64, 64)
    assert pk.msrep_timing_read() == {}


@pytest.mark.parametrize("vt", [0, 1])
def test_csc_tall_matrix_uses_wide_buckets(vt):
    """More than 2^25 rows: over 4096 row buckets of 8192 rows.  A tall
    sparse matrix (rows concentrated at both ends and spread in between)
    checked against the oracle with beta != 0, in both product layouts."""
    rng = np.random.default_rng(13)
    m, n, nnz = (1 << 25) + 4097, 3000, 60_000
    rows = np.concatenate([rng.integers(0, 50_000, nnz // 3), rng.integers(m - 50_000, m, nnz // 3),
                           rng.integers(0, m, nnz - 2 * (nnz // 3))])
    cols = rng.integers(0, n, nnz)
    key = np.unique(rows.astype(np.int64) * n + cols)
    rows, cols = (key // n).astype(np.int64), (key % n).astype(np.int32)
    counts = np.bincount(rows, minlength=m)
    ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    A = synth.Csr(m, n, ptr, cols, rng.uniform(-1, 1, len(cols)), name="tall")
    x = rng.uniform(-1, 1, n)
    y_in = rng.uniform(-1, 1, m)
    tol = F64_TOL if vt == 0 else F32_TOL
    M, v64 = device_mat(A, "csc", vt)
    for np_ in (3, 1000):
        for pf in (1, 2, 3):
            y, ref, s = _run(A, x, "csc", vt, np_, 0.5, 2.0, y_in, M=M, v64=v64,
                             tune=pk.Tune(pipeline=pf))
            assert_close(y, ref, s, tol, "tall csc vt%d np%d pf%d" % (vt, np_, pf))


@pytest.mark.parametrize("vt", [0, 1])
def test_column_merge_taller_than_the_buckets(vt):
    """More than 2^26 rows, beyond the bucketed path's reach: CSC, COO sorted
    by column and COO in any order run the row-window path whatever the
    tune's pipeline (rows spread over the whole height spill to device
    atomics), checked against the oracle with beta != 0; the workspace query
    sizes it, and a prepared call gives the same y."""
    rng = np.random.default_rng(17)
    m, n, nnz = (1 << 26) + 4097, 2000, 40_000
    rows = np.concatenate([rng.integers(0, 30_000, nnz // 2), rng.integers(0, m, nnz - nnz // 2)])
    cols = rng.integers(0, n, nnz)
    key = np.unique(rows.astype(np.int64) * n + cols)
    rows, cols = (key // n).astype(np.int64), (key % n).astype(np.int32)
    ptr = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=m))]).astype(np.int32)
    A = synth.Csr(m, n, ptr, cols, rng.uniform(-1, 1, len(cols)), name="taller")
    x = rng.uniform(-1, 1, n)
    y_in = rng.uniform(-1, 1, m)
    tol = F64_TOL if vt == 0 else F32_TOL
    for fmt in ("csc", "coo_col"):
        M, v64 = device_mat(A, fmt, vt)
        assert pk.msrep_spmv_ws_bytes(M, 7) >= 8 * m
        for pf in (1, 3):
            y, ref, s = _run(A, x, fmt, vt, 7, 0.5, 2.0, y_in, M=M, v64=v64,
                             tune=pk.Tune(pipeline=pf))
            assert_close(y, ref, s, tol, "taller %s vt%d pf%d" % (fmt, vt, pf))
        del M
    # COO in any order: the row-sorted COO shuffled
    from gpu_common import stored_values
    H = host_formats(A)
    r, c, v = H["coo"]
    perm = rng.permutation(len(c))
    sv, v64 = stored_values(v[perm], vt)
    M = pk.Mat(pk.COO_ANY, vt, A.m, A.n, idx=r[perm], idx2=c[perm], val=sv)
    P = pk.msrep_build_partition(M, 5)
    xdt = np.float64 if vt == 0 else np.float32
    xs = torch.from_numpy(x.astype(xdt)).to(_dev())
    y = torch.from_numpy(y_in.astype(xdt)).to(_dev())
    ws = pk.msrep_spmv_prepare(M, P)
    pk.msrep_spmv_prepared(M, P, xs, y, ws, 0.5, 2.0)
    torch.cuda.synchronize()
    ref, s = oracle.spmv_coo(A.m, A.n, r[perm], c[perm], v64, x.astype(xdt).astype(np.float64),
                             0.5, 2.0, y_in.astype(xdt).astype(np.float64))
    assert_close(y.cpu().numpy(), ref, s, tol, "taller coo_any vt%d" % vt)
    del M, P, ws, xs, y
    torch.cuda.empty_cache()


@pytest.mark.parametrize("fmt", FMTS)
def test_spmv_replays_under_graph_capture(fmt):
    """msrep_spmv launches kernels only (no memsets), so a caller can capture
    it: three replays with new x contents, eager work and synchronisation in
    between, each equal to the eager call on the same x."""
    A, x0 = synth.rmat_csr(scale=13, edge_factor=8, seed=21)
    M, v64 = device_mat(A, fmt, pk.F64)
    P = pk.msrep_build_partition(M, 300)
    dev = _dev()
    x = torch.from_numpy(x0).to(dev)
    y = torch.zeros(A.m, dtype=torch.float64, device=dev)
    ws = torch.zeros(pk.msrep_spmv_ws_bytes(M, P.np), dtype=torch.uint8, device=dev)
    pk.msrep_spmv(M, P, x, y, 1.0, 0.0, ws=ws)  # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pk.msrep_spmv(M, P, x, y, 1.0, 0.0, ws=ws)
    rng = np.random.default_rng(22)
    for rep in range(3):
        xn = rng.uniform(-1, 1, A.n)
        x.copy_(torch.from_numpy(xn))
        g.replay()
        torch.cuda.synchronize()
        got = y.cpu().numpy().copy()
        y_eager = torch.zeros_like(y)
        pk.msrep_spmv(M, P, x, y_eager, 1.0, 0.0, ws=torch.zeros_like(ws))
        torch.cuda.synchronize()
        ref, s = oracle_y(A, fmt, v64, xn)
        assert_close(got, ref, s, F64_TOL, "%s replay %d" % (fmt, rep))
        if fmt not in BUCKETED:  # the bucketed path sums in an order that varies
            assert np.array_equal(got, y_eager.cpu().numpy()), (fmt, rep)


@pytest.mark.parametrize("fmt", ["csc", "coo_col", "coo_any"])
@pytest.mark.parametrize("vt", [0, 1, 2])
def test_row_windows_banded_and_spilled(fmt, vt):
    """The windowed column merge (pipeline 3): on stencils the producers'
    rows fit their LDS windows; on R-MAT they do not and the rest goes
    through the spill sums.  Both against the oracle, with alpha and beta,
    for several np; dyadic stencils bit-exact."""
    tol = F64_TOL if vt == 0 else F32_TOL
    rng = np.random.default_rng(41)
    sets = [synth.stencil7_csr(40), synth.rmat_csr(scale=13, edge_factor=16, seed=12),
            synth.uniform_csr(2000, 30000, 9, seed=5)]
    for A, x in sets:
        if fmt == "coo_any":
            M, r, c, v64 = _coo_any(A, vt, 3)
        else:
            M, v64 = device_mat(A, fmt, vt)
        y_in = rng.uniform(-1, 1, A.m)
        for np_ in (1, 37, 2000, A.nnz + 5):
            for alpha, beta in ((1.0, 0.0), (0.5, -2.0)):
                if fmt == "coo_any":
                    xs = np.asarray(x, np.float64 if vt == 0 else np.float32)
                    P = pk.msrep_build_partition(M, np_)
                    yd = torch.from_numpy(y_in.astype(xs.dtype)).to(_dev())
                    pk.msrep_spmv(M, P, torch.from_numpy(xs).to(_dev()), yd, alpha, beta,
                                  pk.Tune(pipeline=3))
                    torch.cuda.synchronize()
                    yi = None if beta == 0.0 else y_in.astype(xs.dtype).astype(np.float64)
                    ref, s = oracle.spmv_coo(A.m, A.n, r, c, v64, xs.astype(np.float64), alpha,
                                             beta, yi)
                    y = yd.cpu().numpy()
                else:
                    y, ref, s = _run(A, x, fmt, vt, np_, alpha, beta, y_in, M=M, v64=v64,
                                     tune=pk.Tune(pipeline=3))
                assert_close(y, ref, s, tol, "%s %s vt%d np%d b%g windows" % (A.name, fmt, vt,
                                                                              np_, beta))
    # dyadic stencil: exact sums in any order
    A, _ = synth.stencil7_csr(32)
    x = synth.dyadic(rng, A.n)
    M, v64 = device_mat(A, "csc" if fmt == "coo_any" else fmt, pk.F64)
    if fmt != "coo_any":
        y, ref, _ = _run(A, x, fmt, pk.F64, 500, M=M, v64=v64, tune=pk.Tune(pipeline=3))
        assert np.array_equal(y, ref)


def test_row_windows_rejected_for_row_formats():
    A, x = synth.uniform_csr(100, 100, 5, seed=1)
    M, _ = device_mat(A, "csr", pk.F64)
    P = pk.msrep_build_partition(M, 4)
    y = torch.zeros(A.m, dtype=torch.float64, device=_dev())
    with pytest.raises(pk.MsrepError) as e:
        pk.msrep_spmv(M, P, torch.from_numpy(x).to(_dev()), y, tune=pk.Tune(pipeline=3))
    assert e.value.status == -1
