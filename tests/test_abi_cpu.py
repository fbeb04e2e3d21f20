"""CPU-only checks of the C ABI: the library loads, exports every function
include/msrep.h declares, its struct layouts agree with the binding, and the
O(1) argument checks fail cleanly without touching a GPU."""
import ctypes
import os

import numpy as np
import pytest

import paper_2209_07552_amd as pk
from paper_2209_07552_amd import _abi


def _lib():
    if not os.path.exists(pk.lib_path()):
        pytest.skip("libmsrep.so not built (python -m paper_2209_07552_amd.build)")
    return pk.load_library()


def test_exports_every_declared_symbol():
    _lib()
    names = _abi.header_functions()
    for must in ("msrep_build_partition", "msrep_convert", "msrep_spmv", "msrep_spmv_batched",
                 "msrep_serve"):
        assert must in names
    missing = [n for n, ok in pk.exported_symbols().items() if not ok]
    assert not missing, missing


def test_struct_sizes():
    assert ctypes.sizeof(_abi._Mat) == 56
    assert pk.PART_DTYPE.itemsize == 40
    assert ctypes.sizeof(_abi._Tune) == 24
    assert ctypes.sizeof(_abi._KernelTime) == 64


def test_lptr_bound_and_vtype_bytes():
    L = _lib()
    assert pk.msrep_lptr_bound(100, 8) == 116
    assert pk.msrep_lptr_bound(0, 1) == 2
    assert pk.msrep_lptr_bound(-1, 8) == -1 and pk.msrep_lptr_bound(5, 0) == -1
    assert [L.msrep_vtype_bytes(v) for v in (0, 1, 2, 9)] == [8, 4, 2, 0]


def _desc(**kw):
    d = dict(fmt=0, vtype=0, m=4, n=4, nnz=4, ptr=0x1000, idx=0x2000, idx2=None, val=0x3000)
    d.update(kw)
    return _abi._Mat(d["fmt"], d["vtype"], d["m"], d["n"], d["nnz"], d["ptr"], d["idx"], d["idx2"],
                     d["val"])


@pytest.mark.parametrize("kw,np_,code", [
    (dict(fmt=7), 4, -1),
    (dict(vtype=5), 4, -1),
    (dict(m=-1), 4, -1),
    (dict(nnz=1 << 31), 4, -3),
    (dict(ptr=None), 4, -1),
    (dict(m=0), 4, -1),            # nonzeros but no rows
    (dict(fmt=2, idx2=None), 4, -1),
    ({}, 0, -1),                   # np <= 0
])
def test_build_partition_argument_errors(kw, np_, code):
    L = _lib()
    d = _desc(**kw)
    st = L.msrep_build_partition(ctypes.byref(d), np_, 0x4000, 0x5000, 1 << 20, None, None)
    assert st == code
    assert L.msrep_last_error()  # a message is set


@pytest.mark.parametrize("kw,np_,code", [
    (dict(fmt=3, idx2=0x6000), 4, -7),  # COO in any order has no row blocks
    ({}, 0, -1),
    (dict(ptr=None), 4, -1),
])
def test_build_partition_rows_argument_errors(kw, np_, code):
    L = _lib()
    d = _desc(**kw)
    st = L.msrep_build_partition_rows(ctypes.byref(d), np_, 0x4000, 0x5000, 1 << 20, None, None)
    assert st == code
    assert L.msrep_last_error()


def test_serve_fill_x_argument_errors():
    from paper_2209_07552_amd import serving
    L = _lib()
    serving._bind(L)
    assert L.msrep_serve_fill_x(0, 1, 0, None, 10, 0, None) == -1   # NULL x with n > 0
    assert L.msrep_serve_fill_x(0, 1, 0, 0x1000, -1, 0, None) == -1  # negative n
    assert L.msrep_serve_fill_x(0, 1, 0, 0x1000, 10, 2, None) == -1  # BF16 vectors do not exist
    assert L.msrep_serve_fill_x(0, 1, 0, None, 0, 0, None) == 0     # empty: nothing launched


def test_spmv_argument_errors():
    L = _lib()
    d = _desc()
    # workspace too small
    st = L.msrep_spmv(ctypes.byref(d), 0x4000, 0x5000, 8, 0x6000, 0x7000, 1.0, 0.0, None, 0x8000,
                      16, None)
    assert st == -3 and b"workspace" in L.msrep_last_error()
    t = _abi._Tune(5, 0, 0, 0, 0, 0)
    st = L.msrep_spmv(ctypes.byref(d), 0x4000, 0x5000, 8, 0x6000, 0x7000, 1.0, 0.0,
                      ctypes.byref(t), 0x8000, 1 << 20, None)
    assert st == -1 and b"k_per_lane" in L.msrep_last_error()
    t = _abi._Tune(4, 4, 2, 0, 0, 0)
    st = L.msrep_spmv(ctypes.byref(d), 0x4000, 0x5000, 8, 0x6000, 0x7000, 1.0, 0.0,
                      ctypes.byref(t), 0x8000, 1 << 20, None)
    assert st == -1 and b"resident" in L.msrep_last_error()
    assert L.msrep_spmv_ws_bytes(ctypes.byref(d), 8) >= 16 * 8
    dc = _desc(fmt=1, vtype=1, m=1000)
    assert L.msrep_spmv_ws_bytes(ctypes.byref(dc), 8) >= 8 * 1000


def test_spmv_prepare_argument_errors():
    """The prepare / prepared split checks its arguments like msrep_spmv,
    before any launch."""
    L = _lib()
    for fmt in (0, 1, 2):
        d = _desc(fmt=fmt, idx2=0x2800 if fmt == 2 else None)
        st = L.msrep_spmv_prepare(ctypes.byref(d), 0x4000, 0x5000, 8, 0x8000, 16, None)
        assert st == -3 and b"msrep_spmv_prepare" in L.msrep_last_error()
        st = L.msrep_spmv_prepare(ctypes.byref(d), 0x4000, 0x5000, 0, 0x8000, 1 << 20, None)
        assert st == -1
        st = L.msrep_spmv_prepared(ctypes.byref(d), 0x4000, 0x5000, 8, None, 0x7000, 1.0, 0.0,
                                   None, 0x8000, 1 << 20, None)
        assert st == -1 and b"x_d" in L.msrep_last_error()
        st = L.msrep_spmv_prepared(ctypes.byref(d), 0x4000, 0x5000, 8, 0x6000, 0x7000, 1.0, 0.0,
                                   None, 0x8000, 16, None)
        assert st == -3 and b"msrep_spmv_prepared" in L.msrep_last_error()


def test_coo_any_order_checks():
    """COO in any order: workspace like CSC, col_idx required; converted from
    (after the workspace check) but never to."""
    L = _lib()
    d = _desc(fmt=3, m=1 << 20, n=1 << 20, nnz=1 << 24, idx2=0x2800)
    assert L.msrep_spmv_ws_bytes(ctypes.byref(d), 16384) >= 12 * (1 << 24)
    bad = _desc(fmt=3, idx2=None)
    st = L.msrep_build_partition(ctypes.byref(bad), 4, 0x4000, None, 0, None, None)
    assert st == -1 and b"idx2" in L.msrep_last_error()
    src = _desc(fmt=3, idx2=0x2800)
    dst = _desc(fmt=0)
    need = L.msrep_convert_ws_bytes(ctypes.byref(src), 0)
    assert need > L.msrep_convert_ws_bytes(ctypes.byref(_desc(fmt=2, idx2=0x2800)), 0)
    st = L.msrep_convert(ctypes.byref(src), ctypes.byref(dst), 0x9000, need - 1, None)
    assert st == -3 and b"workspace" in L.msrep_last_error()
    st = L.msrep_convert(ctypes.byref(_desc(fmt=0)), ctypes.byref(_desc(fmt=3, idx2=0x2800)),
                         0x9000, 1 << 20, None)
    assert st == -7
    big = _desc(fmt=3, m=(1 << 26) + 1, n=4, nnz=4, idx2=0x2800)
    assert L.msrep_spmv_ws_bytes(ctypes.byref(big), 8) >= 8 * ((1 << 26) + 1)  # row windows


def test_csc_workspace_and_row_limit():
    """The CSC path keeps one product and its row offset per nonzero in its
    workspace (room for the 12-byte FP64 / 8-byte FP32 records); its row
    buckets cover m up to 2^26, and taller matrices need only the row-window
    layout (a spill sum per row), so they are sized and accepted too."""
    L = _lib()
    d = _desc(fmt=1, m=1 << 20, n=1 << 20, nnz=1 << 24)
    assert L.msrep_spmv_ws_bytes(ctypes.byref(d), 16384) >= 12 * (1 << 24)
    d32 = _desc(fmt=1, vtype=1, m=1 << 20, n=1 << 20, nnz=1 << 24)
    assert L.msrep_spmv_ws_bytes(ctypes.byref(d32), 16384) >= 8 * (1 << 24)
    big = _desc(fmt=1, m=(1 << 26) + 1, n=4, nnz=4)
    need = L.msrep_spmv_ws_bytes(ctypes.byref(big), 8)
    assert need >= 8 * ((1 << 26) + 1)
    st = L.msrep_spmv(ctypes.byref(big), 0x4000, 0x5000, 8, 0x6000, 0x7000, 1.0, 0.0, None,
                      0x8000, 1 << 20, None)  # checked up to the workspace size, no launch
    assert st == -3 and b"workspace" in L.msrep_last_error()
    ok = _desc(fmt=1, m=1 << 26, n=4, nnz=4)
    assert L.msrep_spmv_ws_bytes(ctypes.byref(ok), 8) > 0


def test_timing_toggle_and_empty_read():
    """Kernel timing is host state: enabling, reading with nothing recorded
    and disabling work without a GPU; a bad buffer is an argument error."""
    L = _lib()
    pk.msrep_timing(True)
    assert pk.msrep_timing_read() == {}
    pk.msrep_timing(False)
    assert L.msrep_timing_read(None, -1) == -1


def test_probe_stream_argument_errors():
    """The stream probe refuses NULL or misaligned buffers, sizes that are
    not whole 16-byte words, unknown modes and overlapping copies, before
    any launch."""
    L = _lib()
    assert L.msrep_probe_stream(None, 0x1000, 4096, 0, 0, None) == -1
    assert L.msrep_probe_stream(0x1008, 0x2000, 4096, 0, 0, None) == -1
    assert L.msrep_probe_stream(0x1000, 0x2000, 4095, 0, 0, None) == -1
    assert L.msrep_probe_stream(0x1000, 0x2000, 0, 1, 0, None) == -1
    assert L.msrep_probe_stream(0x1000, 0x2000, 4096, 2, 0, None) == -1
    assert L.msrep_probe_stream(0x1000, 0x2000, 4096, 0, -1, None) == -1
    assert L.msrep_probe_stream(0x1000, 0x1800, 4096, 1, 0, None) == -1
    assert b"overlap" in L.msrep_last_error()


def test_spmm_argument_errors():
    """msrep_spmm: CSR only, ld >= k, k >= 0, workspace per pass width, all
    checked before any launch."""
    L = _lib()
    d = _desc(fmt=0)
    assert L.msrep_spmm_ws_bytes(ctypes.byref(d), 100, 3) >= 16 * 100 * 3
    assert L.msrep_spmm_ws_bytes(ctypes.byref(d), 100, 20) >= 16 * 100 * 8
    assert L.msrep_spmm_ws_bytes(ctypes.byref(d), 0, 3) == 0
    st = L.msrep_spmm(ctypes.byref(d), 0x4000, 0x5000, 8, 4, 0x6000, 3, 0x7000, 4, 1.0, 0.0,
                      0x8000, 1 << 20, None)
    assert st == -1 and b"ldx" in L.msrep_last_error()
    st = L.msrep_spmm(ctypes.byref(d), 0x4000, 0x5000, 8, -1, 0x6000, 3, 0x7000, 4, 1.0, 0.0,
                      0x8000, 1 << 20, None)
    assert st == -1
    st = L.msrep_spmm(ctypes.byref(d), 0x4000, 0x5000, 8, 4, 0x6000, 4, 0x7000, 4, 1.0, 0.0,
                      0x8000, 16, None)
    assert st == -3 and b"workspace" in L.msrep_last_error()
    for fmt in (1, 2, 3):
        e = _desc(fmt=fmt, idx2=0x2800 if fmt >= 2 else None)
        st = L.msrep_spmm(ctypes.byref(e), 0x4000, 0x5000, 8, 4, 0x6000, 4, 0x7000, 4, 1.0,
                          0.0, 0x8000, 1 << 20, None)
        assert st == -7 and b"CSR" in L.msrep_last_error()
    # k == 0: nothing to do, nothing launched
    st = L.msrep_spmm(ctypes.byref(d), 0x4000, 0x5000, 8, 0, None, 0, None, 0, 1.0, 0.0, None, 0,
                      None)
    assert st == 0
    # Y (m x ldy) or X (n x ldx) of 4 GiB or more: refused before any launch
    big = _desc(fmt=0, m=1 << 26, n=4)
    st = L.msrep_spmm(ctypes.byref(big), 0x4000, 0x5000, 8, 8, 0x6000, 8, 0x7000, 8, 1.0, 0.0,
                      0x8000, 1 << 30, None)
    assert st == -7 and b"4 GiB" in L.msrep_last_error()
    wide = _desc(fmt=0, m=4, n=1 << 26)
    st = L.msrep_spmm(ctypes.byref(wide), 0x4000, 0x5000, 8, 8, 0x6000, 8, 0x7000, 8, 1.0, 0.0,
                      0x8000, 1 << 30, None)
    assert st == -7 and b"4 GiB" in L.msrep_last_error()


@pytest.mark.parametrize("kw,np_,code", [
    (dict(fmt=1), 4, -7),                 # CSC: bucketed path, needs a workspace
    (dict(fmt=3, idx2=0x6000), 4, -7),    # COO in any order likewise
    ({}, 0, -1),
    ({}, (1 << 19) + 1, -3),              # beyond the static scratch
])
def test_spmv_noalloc_argument_errors(kw, np_, code):
    L = _lib()
    d = _desc(**kw)
    assert L.msrep_spmv_noalloc_max_parts() == 1 << 19
    st = L.msrep_spmv_noalloc(ctypes.byref(d), 0x4000, 0x5000, np_, 0x7000, 0x8000, 1.0, 0.0,
                              None, None)
    assert st == code
    assert L.msrep_last_error()


def _cpu_mat(vt=0, m=5, n=4):
    import torch
    ptr = np.zeros(m + 1, np.int32)
    return pk.Mat(pk.CSR, vt, m, n, ptr=ptr, idx=np.zeros(0, np.int32),
                  val=np.zeros(0, np.float64 if vt == 0 else np.float32), device="cpu")


def test_wrappers_reject_bad_vectors():
    """The Python wrappers check x / y / X / Y against the matrix before any
    call reaches the library (the kernels size their buffers from A)."""
    import torch
    A = _cpu_mat()
    P = pk.Partition(A, 1, None, None, None)
    x, y = torch.zeros(4, dtype=torch.float64), torch.zeros(5, dtype=torch.float64)
    bad = [
        (torch.zeros(4, dtype=torch.float32), y, "dtype"),      # FP32 x for F64 values
        (x, torch.zeros(4, dtype=torch.float64), "rows"),       # y shorter than m
        (torch.zeros(3, dtype=torch.float64), y, "rows"),       # x shorter than n
        (torch.zeros(8, dtype=torch.float64)[::2], y, "contiguous"),
        (x, "not a tensor", "tensor"),
    ]
    for fn in (pk.msrep_spmv, pk.msrep_spmv_noalloc, pk.msrep_spmv_prepared):
        for xx, yy, what in bad:
            with pytest.raises((ValueError, TypeError)) as e:
                if fn is pk.msrep_spmv_prepared:
                    fn(A, P, xx, yy, None)
                else:
                    fn(A, P, xx, yy)
            assert what in str(e.value), (fn.__name__, what, str(e.value))
    buf = torch.zeros(9, dtype=torch.float64)
    with pytest.raises(ValueError, match="overlap"):
        pk.msrep_spmv(A, P, buf[:4], buf[3:8])
    # a CPU tensor that is otherwise right is refused as not on the GPU
    with pytest.raises(ValueError, match="GPU"):
        pk.msrep_spmv(A, P, x, y)
    # several right-hand sides
    X, Y = torch.zeros(4, 3, dtype=torch.float64), torch.zeros(5, 3, dtype=torch.float64)
    with pytest.raises(ValueError, match="rows"):
        pk.msrep_spmm(A, P, X, Y[:4])
    with pytest.raises(ValueError, match="dtype"):
        pk.msrep_spmm(A, P, X.float(), Y)
    Z = torch.zeros(9, 3, dtype=torch.float64)
    with pytest.raises(ValueError, match="overlap"):
        pk.msrep_spmm(A, P, Z[:4], Z[2:7])


def test_server_argument_errors():
    """msrep_server_* refuse NULL handles and bad configurations before any
    device call."""
    L = _lib()
    h = ctypes.c_void_p()
    assert L.msrep_server_create(None, None, 0, ctypes.byref(h)) == -1 and not h.value
    cfg = _abi._ServeCfg(0x1000, 1 << 20, 0, 1024, 0, 1.0, 0, 0)  # max_slots 0
    pool = (_abi._HostMat * 1)()
    pool[0].A = _desc()
    assert L.msrep_server_create(ctypes.byref(cfg), pool, 1, ctypes.byref(h)) == -1
    cfg = _abi._ServeCfg(0x1000, 1 << 20, 4, 1024, 0, 1.0, 0, -1)  # negative max_queue
    assert L.msrep_server_create(ctypes.byref(cfg), pool, 1, ctypes.byref(h)) == -1
    for spt in (-1, 65):  # steps_per_tick outside 0..64
        cfg = _abi._ServeCfg(0x1000, 1 << 20, 4, 1024, 0, 1.0, 0, 0, spt)
        assert L.msrep_server_create(ctypes.byref(cfg), pool, 1, ctypes.byref(h)) == -1
        assert b"steps_per_tick" in L.msrep_last_error()
    assert ctypes.sizeof(_abi._ServeCfg) == 56
    r = _abi._Request(0, 0.0, 0, 1)
    assert L.msrep_server_submit(None, ctypes.byref(r), None) == -1
    idx = ctypes.c_int32(7)
    assert L.msrep_server_register(None, pool, ctypes.byref(idx)) == -1
    assert b"NULL" in L.msrep_last_error()
    assert L.msrep_server_poll(None, None, 0, 0) == -1
    assert L.msrep_server_destroy(None, None) == 0
    assert ctypes.sizeof(_abi._Completion) == 40


@pytest.mark.parametrize("vt,vbytes", [(0, 8), (1, 4), (2, 2)])
def test_transposing_conversion_workspace_holds_the_entries(vt, vbytes):
    """A transposing conversion may move whole entries through its sort: its
    workspace has room for every value once more (and the strategy slots);
    conversions that keep the grouping, and COO in any order, do not."""
    L = _lib()
    nnz = 1 << 20
    src = _desc(vtype=vt, m=1000, n=1000, nnz=nnz)
    same = L.msrep_convert_ws_bytes(ctypes.byref(src), 2)      # CSR -> COO
    trans = L.msrep_convert_ws_bytes(ctypes.byref(src), 1)     # CSR -> CSC
    assert trans - same >= vbytes * nnz + 8
    coo = _desc(fmt=2, vtype=vt, m=1000, n=1000, nnz=nnz, idx2=0x2800)
    assert L.msrep_convert_ws_bytes(ctypes.byref(coo), 4) == trans  # COO -> COO_COL transposes
    assert L.msrep_convert_ws_bytes(ctypes.byref(coo), 0) == same   # COO -> CSR does not
