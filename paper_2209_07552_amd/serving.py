"""Binding of msrep_serve / msrep_serve_simulate and of the incremental
server msrep_server_* (argument marshalling only).

A pool entry is a host CSR matrix (ptr, col, val numpy arrays, FP64 or FP32
values).  For msrep_serve the arrays are copied once into pinned host memory
so that uploads into the arena are asynchronous; the arena is one device
tensor of `budget_bytes`.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import _abi
from ._abi import F32, F64, MsrepError, _check, _Completion, _HostMat, _Mat, _Request, _Result, \
    _ServeCfg, _ServeStats, load_library


@dataclass
class ServeResult:
    t_arrive: float
    t_admit: float
    t_done: float
    status: int
    y: Optional[np.ndarray] = None


def _bind(L):
    P = ctypes.POINTER
    f = L.msrep_serve_simulate
    f.restype = ctypes.c_int32
    f.argtypes = [P(_ServeCfg), P(_HostMat), ctypes.c_int32, P(_Request), ctypes.c_int64,
                  P(_Result), P(_ServeStats), ctypes.c_double, ctypes.c_double, ctypes.c_double]
    g = L.msrep_serve_x_value
    g.restype = ctypes.c_double
    g.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64]
    h = L.msrep_serve_fill_x
    h.restype = ctypes.c_int32
    h.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                  ctypes.c_int32, ctypes.c_void_p]


def fill_x(x, seed, rid, step, stream=None):
    """Write x_step of request rid (the server's generator) into the device
    tensor x (FP64 or FP32) on the stream."""
    L = load_library()
    _bind(L)
    vt = F64 if x.dtype == _abi._torch().float64 else F32
    _check(L.msrep_serve_fill_x(int(seed), int(rid), int(step), x.data_ptr(), int(x.numel()), vt,
                                _abi._stream(stream)), "serve_fill_x")
    return x


def x_value(seed, rid, step, c):
    L = load_library()
    _bind(L)
    return float(L.msrep_serve_x_value(seed, rid, step, c))


def _host_pool(pool, vtype, pinned):
    """(array of msrep_host_mat, the host arrays it points into)."""
    keep = []
    hm = (_HostMat * len(pool))()
    vdt = np.float64 if vtype == F64 else np.float32
    for k, A in enumerate(pool):
        ptr = np.ascontiguousarray(A.ptr, np.int32)
        col = np.ascontiguousarray(A.col, np.int32)
        val = np.ascontiguousarray(A.val, vdt)
        if pinned:  # pinned host copies, so that uploads are asynchronous
            import torch
            arrs = [torch.from_numpy(a).pin_memory() for a in (ptr, col, val)]
            keep.extend(arrs)
            pp, cp, vp = (a.data_ptr() for a in arrs)
        else:
            keep.extend((ptr, col, val))
            pp, cp, vp = ptr.ctypes.data, col.ctypes.data, val.ctypes.data
        hm[k].A = _Mat(0, vtype, A.m, A.n, int(ptr[-1]), pp, cp, None, vp)
        hm[k].np = 0
    return hm, keep


@dataclass
class Completion:
    rid: int
    t_arrive: float
    t_admit: float
    t_done: float
    status: int


class Server:
    """The incremental server (msrep_server_create / submit / poll /
    destroy) over a pool of host CSR matrices and a device arena of
    budget_bytes.  Requests are submitted as they come; poll() returns
    completions; close() waits for everything submitted and returns the
    latency statistics."""

    def __init__(self, pool: Sequence, budget_bytes: int, max_slots: int = 256,
                 nnz_per_wave: int = 1024, vtype: int = F64, seed: int = 0, max_queue: int = 0,
                 steps_per_tick: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise MsrepError(-4, "msrep_server needs a GPU")
        self._L = load_library()
        self.pool = list(pool)
        self._hm, self._keep = _host_pool(self.pool, vtype, pinned=True)
        self._arena = torch.empty(int(budget_bytes), dtype=torch.uint8, device="cuda")
        self._cfg = _ServeCfg(self._arena.data_ptr(), int(budget_bytes), int(max_slots),
                              int(nnz_per_wave), int(seed), 1.0, 0, int(max_queue),
                              int(steps_per_tick))
        self.vtype = vtype
        self._ys = {}
        h = ctypes.c_void_p()
        _check(self._L.msrep_server_create(ctypes.byref(self._cfg), self._hm, len(self.pool),
                                           ctypes.byref(h)), "server_create")
        self._h = h.value

    def submit(self, rid: int, matrix: int, steps: int, keep_y: bool = False):
        """Submit request rid (steps SpMVs on pool matrix `matrix`); with
        keep_y its last y is kept (y_of(rid)).  Raises MsrepError with
        status -6 (busy) when the queue is full."""
        y = None
        if keep_y:
            xdt = np.float64 if self.vtype == F64 else np.float32
            y = np.zeros(self.pool[matrix].m, xdt)
            self._ys[int(rid)] = y
        r = _Request(int(rid), 0.0, int(matrix), int(steps))
        _check(self._L.msrep_server_submit(self._h, ctypes.byref(r),
                                           None if y is None else y.ctypes.data), "server_submit")

    def register(self, A) -> int:
        """Add matrix A (synth.Csr or alike) to the running server's pool;
        returns the index requests name it by."""
        hm, keep = _host_pool([A], self.vtype, pinned=True)
        idx = ctypes.c_int32(-1)
        _check(self._L.msrep_server_register(self._h, hm, ctypes.byref(idx)), "server_register")
        self._keep.extend(keep)  # the host arrays stay valid until close()
        self.pool.append(A)
        return int(idx.value)

    def poll(self, cap: int = 1024, timeout_ms: int = 0) -> List[Completion]:
        buf = (_Completion * max(cap, 1))()
        n = self._L.msrep_server_poll(self._h, buf, cap, int(timeout_ms))
        if n < 0:
            raise MsrepError(int(n), _abi.msrep_last_error())
        return [Completion(buf[i].rid, buf[i].t_arrive, buf[i].t_admit, buf[i].t_done,
                           buf[i].status) for i in range(n)]

    def y_of(self, rid: int):
        return self._ys.get(int(rid))

    def close(self) -> dict:
        st = _ServeStats()
        if self._h:
            h, self._h = self._h, None
            _check(self._L.msrep_server_destroy(h, ctypes.byref(st)), "server_destroy")
        return {f: getattr(st, f) for f, _ in _ServeStats._fields_ if not f.startswith("_")}

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serve(pool: Sequence, trace: Sequence, budget_bytes: int, max_slots: int = 256,
          nnz_per_wave: int = 1024, vtype: int = F64, seed: int = 0, time_scale: float = 1.0,
          keep_y: bool = False, simulate: bool = False, sim=(0.0, 0.0, -1.0), nps=None,
          steps_per_tick: int = 0):
    """Run a request trace.  pool: list of synth.Csr (or objects with m, n,
    ptr, col, val); trace: list of synth.Request.  keep_y: True to return
    every request's last y, or a collection of trace indices to return only
    theirs.  steps_per_tick: most steps of one request per tick (0: the
    library's default, 64; a tick runs fewer, in blocks of 8, when the GPU is
    busy, with the same results).  nps: partitions per pool matrix (default:
    nnz_per_wave nonzeros each).  Returns (results, stats)."""
    L = load_library()
    _bind(L)
    keep = []
    hm = (_HostMat * len(pool))()
    vdt = np.float64 if vtype == F64 else np.float32
    xdt = vdt
    torch = None
    if not simulate:
        import torch as _t
        torch = _t
        if not torch.cuda.is_available():
            raise MsrepError(-4, "msrep_serve needs a GPU")
    for k, A in enumerate(pool):
        ptr = np.ascontiguousarray(A.ptr, np.int32)
        col = np.ascontiguousarray(A.col, np.int32)
        val = np.ascontiguousarray(A.val, vdt)
        if torch is not None:  # pinned host copies
            arrs = [torch.from_numpy(a).pin_memory() for a in (ptr, col, val)]
            keep.extend(arrs)
            pp, cp, vp = (a.data_ptr() for a in arrs)
        else:
            keep.extend((ptr, col, val))
            pp, cp, vp = ptr.ctypes.data, col.ctypes.data, val.ctypes.data
        hm[k].A = _Mat(0, vtype, A.m, A.n, int(ptr[-1]), pp, cp, None, vp)
        hm[k].np = 0 if nps is None else int(nps[k])
    n = len(trace)
    tr = (_Request * max(n, 1))()
    for i, r in enumerate(trace):
        tr[i] = _Request(r.rid, r.t_arrive, r.matrix, r.steps)
    res = (_Result * max(n, 1))()
    ybufs = [None] * n
    if keep_y:
        want = range(n) if keep_y is True else sorted(set(int(i) for i in keep_y))
        for i in want:
            ybufs[i] = np.zeros(pool[trace[i].matrix].m, xdt)
            res[i].y_host = ybufs[i].ctypes.data
    arena = None
    if not simulate:
        arena = torch.empty(int(budget_bytes), dtype=torch.uint8, device="cuda")
    cfg = _ServeCfg(None if arena is None else arena.data_ptr(), int(budget_bytes), int(max_slots),
                    int(nnz_per_wave), int(seed), float(time_scale), int(bool(keep_y)), 0,
                    int(steps_per_tick))
    st = _ServeStats()
    if simulate:
        rc = L.msrep_serve_simulate(ctypes.byref(cfg), hm, len(pool), tr, n, res,
                                    ctypes.byref(st), float(sim[0]), float(sim[1]), float(sim[2]))
    else:
        rc = L.msrep_serve(ctypes.byref(cfg), hm, len(pool), tr, n, res, ctypes.byref(st))
    _check(rc, "serve")
    out: List[ServeResult] = []
    for i in range(n):
        out.append(ServeResult(res[i].t_arrive, res[i].t_admit, res[i].t_done, res[i].status,
                               ybufs[i]))
    stats = {f: getattr(st, f) for f, _ in _ServeStats._fields_ if not f.startswith("_")}
    del keep
    return out, stats
