"""ctypes marshalling for libmsrep (include/msrep.h).  Argument marshalling
only: device memory comes from torch tensors, streams from torch.cuda."""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
# MSREP_LIB selects another build of the library (the sanitizer build of
# build.py --sanitize); by default the one next to this file.
_LIB_PATH = os.environ.get("MSREP_LIB") or os.path.join(HERE, "libmsrep.so")
HEADER = os.path.join(ROOT, "include", "msrep.h")

CSR, CSC, COO, COO_ANY, COO_COL = 0, 1, 2, 3, 4  # COO_ANY: any order; COO_COL: by column
COO_FORMATS = (COO, COO_ANY, COO_COL)
F64, F32, BF16 = 0, 1, 2
FMT_NAMES = {CSR: "csr", CSC: "csc", COO: "coo", COO_ANY: "coo_any", COO_COL: "coo_col"}
VT_NAMES = {F64: "f64", F32: "f32", BF16: "bf16"}
VALUE_BYTES = {F64: 8, F32: 4, BF16: 2}

c_i32, c_i64, c_dbl, c_vp, c_sz = (ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                   ctypes.c_void_p, ctypes.c_size_t)


class MsrepError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("msrep status %d: %s" % (status, msg))
        self.status = status


class _Mat(ctypes.Structure):
    _fields_ = [("fmt", c_i32), ("vtype", c_i32), ("m", c_i32), ("n", c_i32), ("nnz", c_i64),
                ("ptr", c_vp), ("idx", c_vp), ("idx2", c_vp), ("val", c_vp)]


class _Tune(ctypes.Structure):
    _fields_ = [("k_per_lane", c_i32), ("waves_per_wg", c_i32), ("resident", c_i32),
                ("nnz_per_wave", c_i32), ("pipeline", c_i32), ("_pad", c_i32)]


class _HostMat(ctypes.Structure):
    _fields_ = [("A", _Mat), ("np", c_i32), ("_pad", c_i32)]


class _ServeCfg(ctypes.Structure):
    _fields_ = [("arena_d", c_vp), ("budget_bytes", c_sz), ("max_slots", c_i32),
                ("nnz_per_wave", c_i32), ("seed", ctypes.c_uint64), ("time_scale", c_dbl),
                ("keep_y", c_i32), ("max_queue", c_i32), ("steps_per_tick", c_i32),
                ("_pad", c_i32)]


class _Request(ctypes.Structure):
    _fields_ = [("rid", c_i64), ("t_arrive", c_dbl), ("matrix", c_i32), ("steps", c_i32)]


class _Result(ctypes.Structure):
    _fields_ = [("t_arrive", c_dbl), ("t_admit", c_dbl), ("t_done", c_dbl), ("status", c_i32),
                ("_pad", c_i32), ("y_host", c_vp)]


class _Completion(ctypes.Structure):
    _fields_ = [("rid", c_i64), ("t_arrive", c_dbl), ("t_admit", c_dbl), ("t_done", c_dbl),
                ("status", c_i32), ("_pad", c_i32)]


class _ServeStats(ctypes.Structure):
    _fields_ = [("p50_ms", c_dbl), ("p99_ms", c_dbl), ("mean_ms", c_dbl), ("max_ms", c_dbl),
                ("req_per_s", c_dbl), ("spmv_per_s", c_dbl), ("makespan_s", c_dbl),
                ("gflops", c_dbl), ("n_done", c_i64), ("n_failed", c_i64), ("ticks", c_i64),
                ("peak_bytes", c_i64), ("peak_active", c_i32), ("_pad", c_i32)]


class _KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("calls", c_i64), ("total_ms", c_dbl)]


PART_DTYPE = np.dtype([("start_idx", "<i8"), ("end_idx", "<i8"), ("start_row", "<i4"),
                       ("end_row", "<i4"), ("start_flag", "<i4"), ("end_flag", "<i4"),
                       ("lptr_off", "<i8")])
assert PART_DTYPE.itemsize == 40

_lib = None


def lib_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libmsrep.so (built by paper_2209_07552_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise MsrepError(-4, "libmsrep.so is not built (python -m paper_2209_07552_amd.build)")
    # torch brings a HIP runtime of its own into the process; it sets up the
    # device before the library's first HIP call (loaded first, the library's
    # runtime has found no device on some hosts)
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except ImportError:
        pass
    L = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    sig = {
        "msrep_last_error": (ctypes.c_char_p, []),
        "msrep_vtype_bytes": (c_i32, [c_i32]),
        "msrep_validate": (c_i32, [P(_Mat), c_vp]),
        "msrep_lptr_bound": (c_i64, [c_i32, c_i32]),
        "msrep_build_partition": (c_i32, [P(_Mat), c_i32, c_vp, c_vp, c_i64, c_vp, c_vp]),
        "msrep_build_partition_rows": (c_i32, [P(_Mat), c_i32, c_vp, c_vp, c_i64, c_vp, c_vp]),
        "msrep_convert_ws_bytes": (c_sz, [P(_Mat), c_i32]),
        "msrep_convert": (c_i32, [P(_Mat), P(_Mat), c_vp, c_sz, c_vp]),
        "msrep_spmv_ws_bytes": (c_sz, [P(_Mat), c_i32]),
        "msrep_spmv": (c_i32, [P(_Mat), c_vp, c_vp, c_i32, c_vp, c_vp, c_dbl, c_dbl, P(_Tune),
                               c_vp, c_sz, c_vp]),
        "msrep_spmv_noalloc_max_parts": (c_i32, []),
        "msrep_spmv_noalloc": (c_i32, [P(_Mat), c_vp, c_vp, c_i32, c_vp, c_vp, c_dbl, c_dbl,
                                       P(_Tune), c_vp]),
        "msrep_spmv_prepare": (c_i32, [P(_Mat), c_vp, c_vp, c_i32, c_vp, c_sz, c_vp]),
        "msrep_spmv_prepared": (c_i32, [P(_Mat), c_vp, c_vp, c_i32, c_vp, c_vp, c_dbl, c_dbl,
                                        P(_Tune), c_vp, c_sz, c_vp]),
        "msrep_spmm_ws_bytes": (c_sz, [P(_Mat), c_i32, c_i32]),
        "msrep_spmm": (c_i32, [P(_Mat), c_vp, c_vp, c_i32, c_i32, c_vp, c_i64, c_vp, c_i64,
                               c_dbl, c_dbl, c_vp, c_sz, c_vp]),
        "msrep_autotune_ws_bytes": (c_sz, [P(_Mat)]),
        "msrep_autotune": (c_i32, [P(_Mat), c_vp, c_vp, c_sz, P(_Tune), c_vp]),
        "msrep_plan_ws_bytes": (c_sz, [c_i32, P(_Mat), P(_Tune)]),
        "msrep_plan_create": (c_i32, [c_i32, P(_Mat), P(_Tune), c_dbl, c_dbl, c_vp, c_sz, c_vp,
                                      P(c_vp)]),
        "msrep_spmv_batched": (c_i32, [c_vp, P(c_vp), P(c_vp), c_vp]),
        "msrep_plan_items": (c_i64, [c_vp]),
        "msrep_plan_destroy": (c_i32, [c_vp]),
        "msrep_serve": (c_i32, [P(_ServeCfg), P(_HostMat), c_i32, P(_Request), c_i64, P(_Result),
                                P(_ServeStats)]),
        "msrep_server_create": (c_i32, [P(_ServeCfg), P(_HostMat), c_i32, P(c_vp)]),
        "msrep_server_submit": (c_i32, [c_vp, P(_Request), c_vp]),
        "msrep_server_register": (c_i32, [c_vp, P(_HostMat), P(c_i32)]),
        "msrep_server_poll": (c_i64, [c_vp, P(_Completion), c_i64, c_i32]),
        "msrep_server_destroy": (c_i32, [c_vp, P(_ServeStats)]),
        "msrep_timing": (c_i32, [c_i32]),
        "msrep_timing_only": (c_i32, [ctypes.c_char_p]),
        "msrep_timing_read": (c_i32, [P(_KernelTime), c_i32]),
        "msrep_probe_stream": (c_i32, [c_vp, c_vp, c_sz, c_i32, c_i32, c_vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def header_functions() -> list:
    """Names of the functions include/msrep.h declares."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(msrep_[a-z0-9_]+)\s*\(", src)))


def exported_symbols() -> dict:
    """{name: bool} -- whether libmsrep.so exports each declared function."""
    L = load_library()
    out = {}
    for name in header_functions():
        try:
            getattr(L, name)
            out[name] = True
        except AttributeError:
            out[name] = False
    return out


def msrep_last_error() -> str:
    return load_library().msrep_last_error().decode()


def _check(st, what=""):
    if st != 0:
        raise MsrepError(st, msrep_last_error() or what)


def msrep_lptr_bound(rows: int, np_: int) -> int:
    return int(load_library().msrep_lptr_bound(rows, np_))


# ------------------------------------------------------------------ torch glue
def _torch():
    import torch
    return torch


def _require_gpu():
    torch = _torch()
    if not torch.cuda.is_available():
        raise MsrepError(-4, "no HIP device available: libmsrep needs an MI355X")
    load_library()
    return torch


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return c_vp(s.cuda_stream)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _dev(a, dtype, device):
    """numpy / torch array -> contiguous torch tensor on device (no copy if it
    already is one)."""
    torch = _torch()
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        t = a
        if t.dtype != dtype:
            raise TypeError("expected %s, got %s" % (dtype, t.dtype))
        return t.to(device).contiguous()
    arr = np.ascontiguousarray(a)
    np_dtype = {torch.int32: np.int32, torch.float64: np.float64, torch.float32: np.float32,
                torch.int16: np.int16}[dtype]
    if arr.dtype == np.uint16 and np_dtype == np.int16:
        arr = arr.view(np.int16)
    return torch.from_numpy(np.ascontiguousarray(arr, dtype=np_dtype)).to(device)


def value_dtype(vtype):
    torch = _torch()
    return {F64: torch.float64, F32: torch.float32, BF16: torch.int16}[vtype]


def vector_dtype(vtype):
    torch = _torch()
    return torch.float64 if vtype == F64 else torch.float32


class Mat:
    """A matrix in device memory plus its C descriptor.  BF16 values are kept
    as raw 16-bit patterns in an int16 tensor."""

    def __init__(self, fmt, vtype, m, n, ptr=None, idx=None, idx2=None, val=None, device="cuda"):
        torch = _torch()
        self.fmt, self.vtype, self.m, self.n = int(fmt), int(vtype), int(m), int(n)
        self.ptr = _dev(ptr, torch.int32, device)
        self.idx = _dev(idx, torch.int32, device)
        self.idx2 = _dev(idx2, torch.int32, device)
        self.val = _dev(val, value_dtype(vtype), device)
        self.nnz = 0 if self.idx is None else int(self.idx.numel())

    @classmethod
    def empty(cls, fmt, vtype, m, n, nnz, device="cuda"):
        torch = _torch()
        M = cls.__new__(cls)
        M.fmt, M.vtype, M.m, M.n, M.nnz = int(fmt), int(vtype), int(m), int(n), int(nnz)
        major = n if fmt == CSC else m
        M.ptr = None if fmt in COO_FORMATS else torch.empty(major + 1, dtype=torch.int32,
                                                            device=device)
        M.idx = torch.empty(nnz, dtype=torch.int32, device=device)
        M.idx2 = (torch.empty(nnz, dtype=torch.int32, device=device) if fmt in COO_FORMATS
                  else None)
        M.val = torch.empty(nnz, dtype=value_dtype(vtype), device=device)
        return M

    def desc(self) -> _Mat:
        return _Mat(self.fmt, self.vtype, self.m, self.n, self.nnz, _ptr(self.ptr), _ptr(self.idx),
                    _ptr(self.idx2), _ptr(self.val))

    @property
    def major(self):
        return self.n if self.fmt in (CSC, COO_COL) else self.m

    def nbytes(self):
        return sum(t.numel() * t.element_size() for t in (self.ptr, self.idx, self.idx2, self.val)
                   if t is not None)


def mat_from_csr(ptr, col, val, m, n, vtype=F64, device="cuda"):
    return Mat(CSR, vtype, m, n, ptr=ptr, idx=col, val=val, device=device)


@dataclass
class Tune:
    k_per_lane: int = 0
    waves_per_wg: int = 0
    resident: int = 0
    nnz_per_wave: int = 0
    pipeline: int = 0

    def c(self) -> _Tune:
        return _Tune(self.k_per_lane, self.waves_per_wg, self.resident, self.nnz_per_wave,
                     self.pipeline, 0)


class Partition:
    """np partitions on the device: ``parts`` (np x 40 bytes) and ``lptr``."""

    def __init__(self, A: Mat, np_: int, parts, lptr, lptr_len):
        self.A, self.np, self.parts, self.lptr, self.lptr_len = A, int(np_), parts, lptr, lptr_len

    def host(self):
        """(structured numpy array of the np records, lptr numpy array)."""
        rec = self.parts.cpu().numpy().view(PART_DTYPE).reshape(-1)
        lp = self.lptr.cpu().numpy() if self.lptr is not None else np.zeros(0, np.int32)
        return rec, lp


def msrep_validate(A: Mat, stream=None):
    _require_gpu()
    d = A.desc()
    _check(load_library().msrep_validate(ctypes.byref(d), _stream(stream)), "validate")


SPLIT_NNZ, SPLIT_ROWS = 0, 1  # equal-nnz partitions / the paper's equal-rows Baseline


def msrep_build_partition(A: Mat, np_: int, stream=None, split: int = SPLIT_NNZ) -> Partition:
    """np_ equal-nnz partitions of A (split=SPLIT_ROWS: the Baseline's equal
    row blocks, msrep_build_partition_rows)."""
    torch = _require_gpu()
    L = load_library()
    dev = A.idx.device if A.idx is not None else A.ptr.device
    parts = torch.empty(max(np_, 1) * PART_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    if A.fmt in COO_FORMATS:
        lptr, cap = None, 0
    else:
        cap = L.msrep_lptr_bound(A.major, np_)
        if cap < 0:
            raise MsrepError(-1, "bad rows/np")
        lptr = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    ln = torch.zeros(1, dtype=torch.int64, device=dev)
    d = A.desc()
    fn = L.msrep_build_partition_rows if split == SPLIT_ROWS else L.msrep_build_partition
    _check(fn(ctypes.byref(d), np_, _ptr(parts), _ptr(lptr), cap, _ptr(ln), _stream(stream)),
           "build_partition")
    return Partition(A, np_, parts, lptr, ln)


_ws_cache = {}


def _workspace(nbytes, device, stream=None):
    """A cached scratch tensor per (device, stream): calls on one stream are
    ordered, so they may share it; another stream gets its own."""
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream(device)
    key = (str(device), int(s.cuda_stream))
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        if stream is not None:
            buf.record_stream(stream)
        _ws_cache[key] = buf
    return buf


def _scratch(nbytes, device, stream=None):
    """A workspace for one call: torch's caching allocator may reuse it once
    the call's work on `stream` (if given) has finished."""
    torch = _torch()
    buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    if stream is not None:
        buf.record_stream(stream)
    return buf


def _span(t, rows, ld, k):
    """Byte range [lo, hi) that rows x k elements of t at row stride ld cover."""
    if rows == 0 or k == 0:
        return (t.data_ptr(), t.data_ptr())
    lo = t.data_ptr()
    return (lo, lo + ((rows - 1) * ld + k) * t.element_size())


def _check_operand_shape(A: Mat, t, name, rows):
    """t is a torch tensor of A's vector dtype with at least `rows` rows."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor on the GPU" % name)
    want = vector_dtype(A.vtype)
    if t.dtype != want:
        raise ValueError("%s has dtype %s; a %s matrix needs %s" % (name, t.dtype,
                                                                    VT_NAMES[A.vtype], want))
    have = t.shape[0] if t.dim() > 0 else 0
    if have < rows:
        raise ValueError("%s has %d rows; the matrix needs %d" % (name, have, rows))


def _check_operand_device(A: Mat, t, name):
    """t is on the GPU that holds A."""
    ref = A.idx if A.idx is not None else A.ptr
    if ref is not None and t.device != ref.device:
        raise ValueError("%s is on %s, the matrix on %s" % (name, t.device, ref.device))
    if not t.is_cuda:
        raise ValueError("%s must be on the GPU" % name)


def _check_operands(A: Mat, X, Y, rows_x, rows_y, ldx, ldy, k, what):
    """Shapes and dtypes first, then overlap of the spans the kernels touch,
    then devices."""
    _check_operand_shape(A, X, what[0], rows_x)
    _check_operand_shape(A, Y, what[1], rows_y)
    xs, ys = _span(X, rows_x, ldx, k), _span(Y, rows_y, ldy, k)
    if xs[0] < ys[1] and ys[0] < xs[1]:
        raise ValueError("%s and %s overlap" % what)
    _check_operand_device(A, X, what[0])
    _check_operand_device(A, Y, what[1])


def _check_vectors(A: Mat, x, y):
    """x (n values) and y (m values) match A: type, dtype, length, unit
    stride, no overlap, device."""
    torch = _torch()
    for t, name in ((x, "x"), (y, "y")):
        if isinstance(t, torch.Tensor) and (t.dim() != 1 or (t.numel() > 1 and t.stride(0) != 1)):
            raise ValueError("%s must be a contiguous 1-D tensor" % name)
    _check_operands(A, x, y, A.n, A.m, 1, 1, 1, ("x", "y"))


def msrep_timing(enable: bool) -> None:
    """Turn per-kernel event timing of msrep_spmv on or off (discards what
    was recorded)."""
    _check(load_library().msrep_timing(1 if enable else 0), "timing")


def msrep_timing_only(kernel: Optional[str] = None) -> None:
    """Time only the kernel of this name (None: every kernel)."""
    _check(load_library().msrep_timing_only(kernel.encode() if kernel else None), "timing_only")


def msrep_timing_read() -> dict:
    """{kernel name: (launches, total ms)} recorded since the last read."""
    L = load_library()
    buf = (_KernelTime * 64)()
    n = L.msrep_timing_read(buf, 64)
    if n < 0:
        raise MsrepError(n, msrep_last_error() or "timing read")
    return {buf[i].name.decode(): (int(buf[i].calls), float(buf[i].total_ms))
            for i in range(min(n, 64))}


def msrep_probe_stream(src, dst, mode: int, blocks: int = 0, stream=None) -> None:
    """Launch the plain stream probe over all of src (mode 0: read, with dst
    a 16-byte sink; mode 1: copy into dst of the same size)."""
    nbytes = src.numel() * src.element_size()
    _check(load_library().msrep_probe_stream(_ptr(src), _ptr(dst), nbytes, int(mode), int(blocks),
                                             _stream(stream)), "probe_stream")


def msrep_spmv_ws_bytes(A: Mat, np_: int) -> int:
    """Bytes of device workspace msrep_spmv needs for A split into np_ parts."""
    return int(load_library().msrep_spmv_ws_bytes(ctypes.byref(A.desc()), int(np_)))


def msrep_spmv(A: Mat, P: Partition, x, y, alpha=1.0, beta=0.0, tune: Optional[Tune] = None,
               ws=None, stream=None):
    """y <- alpha*A*x + beta*y (in place on the device tensor y); returns y."""
    _check_vectors(A, x, y)
    _require_gpu()
    L = load_library()
    d = A.desc()
    need = L.msrep_spmv_ws_bytes(ctypes.byref(d), P.np)
    if ws is None:
        ws = _workspace(need, y.device, stream)
    t = tune.c() if tune is not None else None
    _check(L.msrep_spmv(ctypes.byref(d), _ptr(P.parts), _ptr(P.lptr), P.np, _ptr(x), _ptr(y),
                        float(alpha), float(beta), ctypes.byref(t) if t is not None else None,
                        _ptr(ws), ws.numel(), _stream(stream)), "spmv")
    return y


def msrep_spmv_noalloc_max_parts() -> int:
    """Most partitions msrep_spmv_noalloc takes (its static scratch)."""
    return int(load_library().msrep_spmv_noalloc_max_parts())


def msrep_spmv_noalloc(A: Mat, P: Partition, x, y, alpha=1.0, beta=0.0,
                       tune: Optional[Tune] = None, stream=None):
    """msrep_spmv for CSR / row-sorted COO with the boundary carries in the
    library's static device scratch (no workspace); returns y."""
    _check_vectors(A, x, y)
    _require_gpu()
    L = load_library()
    d = A.desc()
    t = tune.c() if tune is not None else None
    _check(L.msrep_spmv_noalloc(ctypes.byref(d), _ptr(P.parts), _ptr(P.lptr), P.np, _ptr(x),
                                _ptr(y), float(alpha), float(beta),
                                ctypes.byref(t) if t is not None else None, _stream(stream)),
           "spmv_noalloc")
    return y


def msrep_spmv_prepare(A: Mat, P: Partition, ws=None, stream=None):
    """The structure-only part of msrep_spmv (CSC: bucket counts, offsets and
    pieces) into the workspace ws (a new one of its own if None, never the
    shared cache that msrep_spmv uses); returns ws, to be passed to
    msrep_spmv_prepared with the same A structure, P and np."""
    torch = _require_gpu()
    L = load_library()
    d = A.desc()
    need = L.msrep_spmv_ws_bytes(ctypes.byref(d), P.np)
    if ws is None:
        ws = _scratch(need, P.parts.device, stream)
    _check(L.msrep_spmv_prepare(ctypes.byref(d), _ptr(P.parts), _ptr(P.lptr), P.np, _ptr(ws),
                                ws.numel(), _stream(stream)), "spmv_prepare")
    return ws


def msrep_spmv_prepared(A: Mat, P: Partition, x, y, ws, alpha=1.0, beta=0.0,
                        tune: Optional[Tune] = None, stream=None):
    """msrep_spmv with ws prepared by msrep_spmv_prepare(A, P); returns y."""
    _check_vectors(A, x, y)
    _require_gpu()
    L = load_library()
    d = A.desc()
    t = tune.c() if tune is not None else None
    _check(L.msrep_spmv_prepared(ctypes.byref(d), _ptr(P.parts), _ptr(P.lptr), P.np, _ptr(x),
                                 _ptr(y), float(alpha), float(beta),
                                 ctypes.byref(t) if t is not None else None, _ptr(ws),
                                 ws.numel(), _stream(stream)), "spmv_prepared")
    return y


def msrep_spmm_ws_bytes(A: Mat, np_: int, k: int) -> int:
    """Bytes of device workspace msrep_spmm needs for k right-hand sides."""
    return int(load_library().msrep_spmm_ws_bytes(ctypes.byref(A.desc()), int(np_), int(k)))


def msrep_spmm(A: Mat, P: Partition, X, Y, alpha=1.0, beta=0.0, ws=None, stream=None):
    """Y <- alpha*A*X + beta*Y for the k columns of the row-major device
    tensors X (n x k) and Y (m x k, updated in place; both may be column
    slices of wider tensors, rows strided by their stride(0)); returns Y."""
    torch = _torch()
    d = A.desc()
    if X.dim() != 2 or Y.dim() != 2 or X.shape[1] != Y.shape[1]:
        raise ValueError("X and Y must be 2-D with the same number of columns")
    if X.stride(1) != 1 or Y.stride(1) != 1:
        raise ValueError("X and Y must have unit column stride (row-major)")
    k = int(X.shape[1])
    _check_operands(A, X, Y, A.n, A.m, int(X.stride(0)), int(Y.stride(0)), k, ("X", "Y"))
    _require_gpu()
    L = load_library()
    need = L.msrep_spmm_ws_bytes(ctypes.byref(d), P.np, k)
    if ws is None:
        ws = _scratch(need, Y.device, stream)
    _check(L.msrep_spmm(ctypes.byref(d), _ptr(P.parts), _ptr(P.lptr), P.np, k, _ptr(X),
                        int(X.stride(0)), _ptr(Y), int(Y.stride(0)), float(alpha), float(beta),
                        _ptr(ws), ws.numel(), _stream(stream)), "spmm")
    return Y


def msrep_convert(A: Mat, dst_fmt: int, stream=None) -> Mat:
    torch = _require_gpu()
    L = load_library()
    dev = A.idx.device if A.idx is not None else A.ptr.device
    B = Mat.empty(dst_fmt, A.vtype, A.m, A.n, A.nnz, device=dev)
    ds, dd = A.desc(), B.desc()
    need = L.msrep_convert_ws_bytes(ctypes.byref(ds), dst_fmt)
    ws = _scratch(need, dev, stream)
    _check(L.msrep_convert(ctypes.byref(ds), ctypes.byref(dd), _ptr(ws), ws.numel(),
                           _stream(stream)), "convert")
    return B


def msrep_autotune(A: Mat, x, stream=None) -> Tune:
    torch = _require_gpu()
    L = load_library()
    d = A.desc()
    need = L.msrep_autotune_ws_bytes(ctypes.byref(d))
    ws = _scratch(need, x.device, stream)
    out = _Tune()
    _check(L.msrep_autotune(ctypes.byref(d), _ptr(x), _ptr(ws), ws.numel(), ctypes.byref(out),
                            _stream(stream)), "autotune")
    return Tune(out.k_per_lane, out.waves_per_wg, out.resident, out.nnz_per_wave, out.pipeline)


class Plan:
    """A batched plan (msrep_plan_create); keeps its workspace alive."""

    def __init__(self, handle, ws, mats, count):
        self.handle, self.ws, self.mats, self.count = handle, ws, mats, count

    def items(self):
        return int(load_library().msrep_plan_items(self.handle))

    def destroy(self):
        if self.handle:
            _check(load_library().msrep_plan_destroy(self.handle), "plan_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def msrep_plan_create(mats: Sequence[Mat], tunes=None, alpha=1.0, beta=0.0, stream=None) -> Plan:
    torch = _require_gpu()
    L = load_library()
    count = len(mats)
    descs = (_Mat * count)(*[M.desc() for M in mats])
    tarr = None
    if tunes is not None:
        tarr = (_Tune * count)(*[(t or Tune()).c() for t in tunes])
    need = L.msrep_plan_ws_bytes(count, descs, tarr)
    ws = torch.empty(max(int(need), 256), dtype=torch.uint8, device=mats[0].idx.device)
    h = c_vp()
    _check(L.msrep_plan_create(count, descs, tarr, float(alpha), float(beta), _ptr(ws), ws.numel(),
                               _stream(stream), ctypes.byref(h)), "plan_create")
    return Plan(h.value, ws, list(mats), count)


def msrep_spmv_batched(plan: Plan, xs, ys, stream=None):
    _require_gpu()
    L = load_library()
    if len(xs) != plan.count or len(ys) != plan.count:
        raise ValueError("plan has %d matrices; got %d x and %d y tensors"
                         % (plan.count, len(xs), len(ys)))
    for i, (M, x, y) in enumerate(zip(plan.mats, xs, ys)):
        try:
            _check_vectors(M, x, y)
        except (TypeError, ValueError) as e:
            raise type(e)("matrix %d: %s" % (i, e)) from None
    xa = (c_vp * plan.count)(*[x.data_ptr() for x in xs])
    ya = (c_vp * plan.count)(*[y.data_ptr() for y in ys])
    _check(L.msrep_spmv_batched(plan.handle, xa, ya, _stream(stream)), "spmv_batched")


def msrep_serve(*args, **kwargs):
    from .serving import serve
    return serve(*args, **kwargs)
