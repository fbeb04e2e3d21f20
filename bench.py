#!/usr/bin/env python3
"""Benchmark of the equal-nnz partitioned SpMV (msRep, arXiv 2209.07552) on
one MI355X.

Default workload: the 3-D 7-point Laplacian on a 256^3 grid in FP64
(16,777,216 rows, 117,047,296 nonzeros, diagonal 6, neighbours -1, x ~
U(-1, 1), seed 0) stored as CSR, CSC and COO, each split into equal-nnz
partitions over the CUs.  One step is y = A*x in each of the three formats
(partitions and matrices resident in HBM, boundary merges included).  The
same line carries the same step with FP32 and BF16 stored values
("precision") and on the power-law R-MAT scale-20 matrix (1,048,576 rows,
edge factor 16, a/b/c/d = .57/.19/.19/.05, duplicates merged; "rmat20"),
every result checked against the FP64 oracle.  Every SpMV of the timed region
runs cache-cold: a 512 MiB scrub write between SpMVs evicts the 256 MB
Infinity Cache, and HIP events on the library's stream bracket each SpMV, so
the reported throughput is the SpMV time alone.  A warm (back-to-back) figure
is reported beside it.

Prints one JSON line (rank 0, N = 1).  --gpus N > 1 exits: the benchmark runs on
one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Launch shape per workload and format used unless --autotune or explicit
# --nnz-per-wave/--k/--wpb/--pipeline/--resident are given: the tuner's picks
# on MI355X (nnz_per_wave, k_per_lane, waves_per_wg, pipeline, resident).
DEFAULT_TUNES = {
    "rmat20": {"csr": (512, 4, 8, 2, 1), "coo": (512, 4, 8, 2, 1), "csc": (1024, 4, 2, 1, 0),
               "coo_any": (1024, 4, 2, 1, 0), "coo_col": (1024, 4, 2, 1, 0)},
    "stencil256": {"csr": (2048, 4, 4, 2, 0), "coo": (1024, 4, 2, 2, 0),
                   "csc": (1024, 4, 2, 3, 0), "coo_any": (1024, 4, 2, 2, 0),
                   "coo_col": (1024, 4, 2, 3, 0)},
}
SCRUB_BYTES = 512 << 20


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_formats(A, any_order=False):
    """CSC, row-sorted COO and column-sorted COO arrays of a CSR matrix
    (plain numpy input preparation: stable sort by column), and with
    any_order the COO in a seeded random order."""
    rows = np.repeat(np.arange(A.m, dtype=np.int32), np.diff(A.ptr))
    perm = np.argsort(A.col, kind="stable")
    cptr = np.zeros(A.n + 1, np.int64)
    np.cumsum(np.bincount(A.col, minlength=A.n), out=cptr[1:])
    out = {"csr": (A.ptr, A.col, A.val),
           "csc": (cptr.astype(np.int32), rows[perm], A.val[perm]),
           "coo": (rows, A.col, A.val),
           "coo_col": (rows[perm], A.col[perm], A.val[perm])}
    if any_order:  # COO in a seeded random order
        shuf = np.random.default_rng(0).permutation(A.nnz)
        out["coo_any"] = (rows[shuf], A.col[shuf], A.val[shuf])
    return out


def alg_bytes(fmt, m, n, nnz, vbytes, xbytes, beta0=True):
    """Bytes the method must move for one SpMV (values, indices, pointer, x
    read once, y written once; y read too when beta != 0)."""
    b = nnz * (vbytes + 4) + n * xbytes + m * xbytes
    if fmt == "csr":
        b += (m + 1) * 4
    elif fmt == "csc":
        b += (n + 1) * 4
    else:
        b += nnz * 4
    if not beta0:
        b += m * xbytes
    return b


COPY_CAL_BYTES = 256 << 20  # plain copy used to calibrate the byte counters


def kernel_source_hash():
    """Hash of the HIP sources: a stored counter reading is current only while
    the kernels are unchanged."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2209_07552_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(kernel_key):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary (profiles/traffic.txt), or None when there is none or the kernel
    sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    cur = kernel_source_hash()
    for line in open(path):
        line = line.strip()
        if not line.startswith("{"):
            continue
        try:
            rec = json.loads(line)
        except ValueError:
            continue
        if rec.get("key") == kernel_key and rec.get("source_hash") == cur:
            return rec.get("bytes_per_launch")
    return None


def _read_counters(d):
    """{(kernel name, counter): [values per dispatch]} from a rocprofv3
    --pmc ... --output-format csv directory."""
    import csv
    import glob
    out = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            out.setdefault((r["Kernel_Name"], r["Counter_Name"]), []).append(float(r["Counter_Value"]))
    return out


def pmc_summary(fetch_dir, write_dir, kernel, key, command):
    """Turn two counter runs (FETCH_SIZE, WRITE_SIZE, KiB per dispatch) into
    HBM bytes per launch of `kernel`, each counter scaled by what it reads for
    the plain copy of COPY_CAL_BYTES in the same run; append to
    profiles/traffic.txt."""
    out = {}
    for d, ctr in ((fetch_dir, "FETCH_SIZE"), (write_dir, "WRITE_SIZE")):
        c = _read_counters(d)
        kv = [v for (k, n), vs in c.items() if n == ctr and kernel in k for v in vs]
        # the calibration copy is the largest copy of the run (the matrix
        # uploads are many small staged copies)
        cv = [v for (k, n), vs in c.items() if n == ctr and "copy" in k.lower() for v in vs]
        if not kv or not cv:
            raise SystemExit("no %s readings for %s / the copy kernel in %s" % (ctr, kernel, d))
        scale = COPY_CAL_BYTES / (float(max(cv)) * 1024.0)
        out[ctr] = (float(np.median(kv)), float(max(cv)), scale)
    fetch = out["FETCH_SIZE"][0] * 1024.0 * out["FETCH_SIZE"][2]
    write = out["WRITE_SIZE"][0] * 1024.0 * out["WRITE_SIZE"][2]
    rec = {"key": key, "kernel": kernel, "bytes_per_launch": int(fetch + write),
           "fetch_bytes": int(fetch), "write_bytes": int(write),
           "fetch_kib_raw": out["FETCH_SIZE"][0], "write_kib_raw": out["WRITE_SIZE"][0],
           "copy_fetch_kib_raw": out["FETCH_SIZE"][1], "copy_write_kib_raw": out["WRITE_SIZE"][1],
           "fetch_scale": round(out["FETCH_SIZE"][2], 4), "write_scale": round(out["WRITE_SIZE"][2], 4),
           "source_hash": kernel_source_hash(), "command": command}
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    lines = []
    if os.path.exists(path):
        lines = [l for l in open(path) if not (l.startswith("{") and json.loads(l).get("key") == key)]
    if not lines:
        lines = ["# HBM traffic per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE (KiB per\n",
                 "# dispatch), each scaled by its reading for a plain 256 MiB copy in the same run.\n"]
    lines.append(json.dumps(rec) + "\n")
    open(path, "w").writelines(lines)
    print(json.dumps(rec))


def counter_summary(dirs, out_name, kernels, command):
    """Mean per dispatch of every counter of rocprofv3 --pmc runs (one
    directory per pass) for the kernels whose names contain one of
    `kernels`, as a short text table under profiles/."""
    rows = {}
    for d in dirs:
        for (k, ctr), vs in _read_counters(d).items():
            name = k.replace("(anonymous namespace)::", "").split("(")[0]
            if not any(x in name for x in kernels):
                continue
            rows.setdefault(name[:70], {})[ctr] = (float(np.mean(vs)), len(vs))
    lines = ["# rocprofv3 counters, mean per dispatch", "# command: " + command, ""]
    for name, ctrs in sorted(rows.items()):
        lines.append(name)
        for ctr, (v, c) in sorted(ctrs.items()):
            lines.append("    %-40s %18.1f   (%d dispatches)" % (ctr, v, c))
    path = os.path.join(ROOT, "profiles", out_name)
    open(path, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def trace_summary(trace_dir, out_name, command, bench_json=None):
    """Kernel-trace statistics (rocprofv3 --kernel-trace --stats, csv) as a
    short text table under profiles/; with the traced run's own JSON line,
    also its event-measured average for the roofline kernel."""
    import csv
    import glob
    files = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise SystemExit("no kernel_stats.csv under %s" % trace_dir)
    rows = list(csv.DictReader(open(files[0])))
    lines = ["# rocprofv3 kernel statistics", "# command: " + command, "",
             "%-72s %8s %12s %12s %7s" % ("kernel", "calls", "avg_us", "total_us", "pct")]
    for r in rows:
        name = r.get("Name", r.get("KernelName", "")).replace("(anonymous namespace)::", "")
        short = name.split("(")[0][:72]
        lines.append("%-72s %8s %12.2f %12.2f %7.2f" % (
            short, r.get("Calls"), float(r.get("AverageNs", 0)) / 1e3,
            float(r.get("TotalDurationNs", 0)) / 1e3, float(r.get("Percentage", 0))))
    # one kernel runs on several matrices in one command: the per-launch
    # trace split by launch grid (the grid tells the matrices apart)
    traces = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if traces:
        by = {}
        for r in csv.DictReader(open(traces[0])):
            name = r.get("Kernel_Name", "").replace("(anonymous namespace)::", "")
            if "msrep::" not in name:
                continue
            grid = r.get("Grid_Size_X", r.get("Grid_Size", "?"))
            d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            by.setdefault((name.split("(")[0][:60], grid), []).append(d)
        top = sorted(by.items(), key=lambda kv: -sum(kv[1]))
        lines += ["", "# per launch grid (msrep kernels, the %d of %d with the most time): calls,"
                  " average and median us" % (min(40, len(top)), len(top)),
                  "%-60s %10s %8s %12s %12s" % ("kernel", "grid", "calls", "avg_us", "median_us")]
        for (name, grid), ds in top[:40]:
            lines.append("%-60s %10s %8d %12.2f %12.2f" % (name, grid, len(ds), sum(ds) / len(ds),
                                                         float(np.median(ds))))
    if bench_json:
        rec = json.loads(open(bench_json).read().strip().splitlines()[-1])
        rf = rec.get("roofline") or {}
        if rf:
            lines += ["", "# the traced run's bench line: roofline kernel %s, %.2f us per launch by"
                      " HIP events, %.1f GB/s algorithmic (%.4f of %g)" % (
                          rf.get("kernel"), rf.get("kernel_avg_us", float("nan")),
                          rf.get("achieved", float("nan")), rf.get("frac", float("nan")),
                          rf.get("peak", float("nan")))]
        else:
            lines += ["", "# the traced run's bench line: %s %s %s, %s ms per step" % (
                rec.get("metric"), rec.get("value"), rec.get("unit"), rec.get("ms_per_step"))]
        for f, v in rec.get("per_format", {}).items():
            lines.append("#   %s: %s" % (f, json.dumps(v.get("kernels_us", {}))))
    path = os.path.join(ROOT, "profiles", out_name)
    open(path, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def overheads(args, mats, part_ms, prep_ms, cold_ms, kt_all):
    """The paper's overhead breakdown (its partition and merge time figures)
    on one GPU: format conversion from CSR on the GPU, partition build, the
    CSC structure work and the boundary merge, each also as a share of that
    format's SpMV time."""
    import torch
    import paper_2209_07552_amd as pk
    out = {}
    if "csr" in mats:
        for dst, name in ((pk.CSC, "csc"), (pk.COO, "coo")):
            pk.msrep_convert(mats["csr"], dst)  # first launch loads the code
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            B = pk.msrep_convert(mats["csr"], dst)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            del B
            out["convert_csr_to_" + name] = {"ms": round(ms, 4), "pct_of_spmv":
                                             round(100 * ms / cold_ms[name], 1) if name in cold_ms else None}
    for f in cold_ms:
        merge = [t / c for (g, k), (c, t) in kt_all.items() if g == f and k in ("merge_rows", "csc_merge")]
        out[f] = {"partition_ms": round(part_ms[f], 4),
                  "partition_pct_of_spmv": round(100 * part_ms[f] / cold_ms[f], 1),
                  "prepare_ms": round(prep_ms[f], 4),
                  "merge_ms": round(sum(merge), 4),
                  "merge_pct_of_spmv": round(100 * sum(merge) / cold_ms[f], 1)}
    return out


def cpu_baseline(A, x, reps=5):
    """The CPU baseline of the FP64 SpMV on this host, as the measurement plan
    states it: the oracle's plain (uncompensated) CSR row loop, OpenMP
    row-parallel with a static schedule, on every core this process may run
    on and on one core, median of `reps` whole SpMVs each; the oracle's
    compensated (Dot2) mode timed separately on one core.  Same matrix and x
    as the GPU run; the same flop count (2 nnz per SpMV)."""
    import oracle
    oracle.build(force=False)
    cores = len(os.sched_getaffinity(0))

    def med(threads, n_):
        ts = []
        for _ in range(n_):
            t0 = time.perf_counter()
            oracle.spmv_csr_plain(A.m, A.n, A.ptr, A.col, A.val, x, threads=threads)
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))
    med(cores, 1)  # first touch of the arrays
    t_all = med(cores, reps)
    t_one = med(1, reps)
    t0 = time.perf_counter()
    oracle.spmv_csr(A.m, A.n, A.ptr, A.col, A.val, x)
    t_dot2 = time.perf_counter() - t0
    fl = 2.0 * A.nnz
    return {"value": round(fl / t_all / 1e9, 4), "unit": "GFLOP/s", "cores": cores,
            "kind": "oracle",
            "sample": "the whole FP64 CSR SpMV of the same matrix (%d nnz): plain row loop, "
                      "OpenMP static over %d threads, median of %d; also on 1 thread (median of "
                      "%d) and the compensated Dot2 mode on 1 thread (one SpMV)"
                      % (A.nnz, cores, reps, reps),
            "ms_all_cores": round(t_all * 1e3, 3),
            "one_core_gflops": round(fl / t_one / 1e9, 4), "ms_one_core": round(t_one * 1e3, 3),
            "dot2_one_core_gflops": round(fl / t_dot2 / 1e9, 4),
            "ms_dot2_one_core": round(t_dot2 * 1e3, 3)}


def gen_workload(name):
    """(Csr, x, workload description) of a named benchmark matrix."""
    import synth
    t0 = time.time()
    if name == "rmat20":
        A, x64 = synth.rmat_csr(scale=20, edge_factor=16, seed=0)
        wl = {"workload": "rmat-scale20-ef16", "rows": A.m, "cols": A.n, "nnz": A.nnz,
              "abcd": [0.57, 0.19, 0.19, 0.05]}
    elif name == "stencil256":
        A, x64 = synth.stencil7_csr(256, seed=0)
        wl = {"workload": "laplace3d-7pt-256^3", "rows": A.m, "cols": A.n, "nnz": A.nnz}
    else:
        A, x64 = synth.uniform_csr(4096, 4096, 16, seed=0)
        wl = {"workload": "uniform-4096-16perrow", "rows": A.m, "cols": A.n, "nnz": A.nnz}
    log("generated %s in %.1fs" % (wl["workload"], time.time() - t0))
    return A, x64, wl


def stored_values(v, vt):
    """FP64 values as the stored type: FP32 rounded once, BF16 from that FP32
    (round to nearest even), as raw bits."""
    import paper_2209_07552_amd as pk
    import synth
    if vt == pk.F64:
        return v
    v32 = np.asarray(v, np.float32)
    return v32 if vt == pk.F32 else synth.bf16_bits(v32)


def stored_as_f64(sv, vt):
    """Stored values (FP64, FP32 or BF16 bits) back in FP64, exactly."""
    import paper_2209_07552_amd as pk
    if vt == pk.BF16:
        return (np.asarray(sv, np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return np.asarray(sv, np.float64)


def measure_matrix(args, A, x64, wl, wkey, vt, fmts, ref=None):
    """Time one step (one cold SpMV per format in fmts) of matrix A on the
    GPU and check every format's y against the FP64 oracle.

    Returns a dict: step time and GFLOP/s, per-format records (cold time,
    algorithmic GB/s and fraction of HBM peak, partition / prepare time,
    launch shape, per-kernel breakdown, largest error relative to (|A||x|)_i)
    and the roofline record of the dominant kernel, priced at its format's
    algorithmic bytes per SpMV.  ref: the oracle's (y, scale) on the FP64
    values, computed here when None."""
    import torch

    import oracle
    import paper_2209_07552_amd as pk
    dev = torch.device("cuda:0")
    H = host_formats(A, any_order="coo_any" in fmts)
    vbytes = pk._abi.VALUE_BYTES[vt]
    xbytes = 8 if vt == pk.F64 else 4
    vname = pk._abi.VT_NAMES[vt]
    mats = {}
    for f in fmts:
        a, b, v = H[f]
        if f == "csr":
            mats[f] = pk.Mat(pk.CSR, vt, A.m, A.n, ptr=a, idx=b, val=stored_values(v, vt))
        elif f == "csc":
            mats[f] = pk.Mat(pk.CSC, vt, A.m, A.n, ptr=a, idx=b, val=stored_values(v, vt))
        else:
            kind = {"coo_any": pk.COO_ANY, "coo_col": pk.COO_COL}.get(f, pk.COO)
            mats[f] = pk.Mat(kind, vt, A.m, A.n, idx=a, idx2=b, val=stored_values(v, vt))
    del H
    xs = x64 if vt == pk.F64 else x64.astype(np.float32)
    x = torch.from_numpy(xs).to(dev)
    ydt = pk._abi.vector_dtype(vt)
    ys = {f: torch.zeros(A.m, dtype=ydt, device=dev) for f in fmts}
    # launch shape and partition size per format: explicit flags, else the
    # stored picks for this workload, else (or with --autotune) the tuner
    tunes, parts, part_ms = {}, {}, {}
    for f in fmts:
        stored_t = DEFAULT_TUNES.get(wkey, {}).get(f)
        if args.nnz_per_wave:
            tunes[f] = pk.Tune(k_per_lane=args.k, waves_per_wg=args.wpb,
                               nnz_per_wave=args.nnz_per_wave, pipeline=args.pipeline,
                               resident=args.resident)
        elif stored_t and not args.autotune:
            tunes[f] = pk.Tune(k_per_lane=stored_t[1], waves_per_wg=stored_t[2],
                               nnz_per_wave=stored_t[0], pipeline=stored_t[3],
                               resident=stored_t[4])
        else:
            tunes[f] = pk.msrep_autotune(mats[f], x)
            log("tuned %s: %s" % (f, tunes[f]))
        np_f = max(1, -(-A.nnz // tunes[f].nnz_per_wave))
        pk.msrep_build_partition(mats[f], np_f)  # first launches load the code
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        parts[f] = pk.msrep_build_partition(mats[f], np_f)
        e1.record()
        torch.cuda.synchronize()
        part_ms[f] = e0.elapsed_time(e1)
        if args.split == "rows" and f != "coo_any":  # the paper's baseline split, same np
            parts[f] = pk.msrep_build_partition(mats[f], np_f, split=pk.SPLIT_ROWS)
            torch.cuda.synchronize()
    scrub = torch.empty(SCRUB_BYTES, dtype=torch.uint8, device=dev)
    ws = {f: torch.zeros(max(256, pk.msrep_spmv_ws_bytes(mats[f], parts[f].np)), dtype=torch.uint8,
                         device=dev) for f in fmts}

    # the structure-only work (CSC: bucket counts, run offsets, pieces) is
    # done once per matrix and partitioning, like the partition build; the
    # timed SpMVs reuse it (msrep_spmv_prepared).  --unprepared times plain
    # msrep_spmv, which redoes it every call.
    prep_ms = {}
    for f in fmts:
        pk.msrep_spmv_prepare(mats[f], parts[f], ws=ws[f])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        pk.msrep_spmv_prepare(mats[f], parts[f], ws=ws[f])
        e1.record()
        torch.cuda.synchronize()
        prep_ms[f] = e0.elapsed_time(e1)

    def spmv(f):
        if args.unprepared:
            pk.msrep_spmv(mats[f], parts[f], x, ys[f], 1.0, 0.0, tunes[f], ws=ws[f])
        else:
            pk.msrep_spmv_prepared(mats[f], parts[f], x, ys[f], ws[f], 1.0, 0.0, tunes[f])

    def fmt_bytes(f):
        return alg_bytes("coo" if f in ("coo_any", "coo_col") else f, A.m, A.n, A.nnz, vbytes,
                         xbytes)

    def priced_of(kt):
        return {fk: v for fk, v in kt.items() if fk[1] in PRICED_KERNELS}

    def timed_steps(steps, only=None):
        """steps cold steps; each SpMV bracketed by events.  only=None: the
        library times every kernel; only=(fmt, kernel): just that kernel in
        that format's SpMV (one event pair, so the step is barely
        perturbed)."""
        ev = {f: [] for f in fmts}
        kt = {}
        for _ in range(steps):
            for f in fmts:
                scrub.fill_(1)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                on = only is None or (only and only[0] == f)
                pk.msrep_timing(on)
                pk.msrep_timing_only(only[1] if only else None)
                e0.record()
                spmv(f)
                e1.record()
                if on:
                    for k, (c, t) in pk.msrep_timing_read().items():
                        kc, ktt = kt.get((f, k), (0, 0.0))
                        kt[(f, k)] = (kc + c, ktt + t)
                ev[f].append((e0, e1))
        pk.msrep_timing(False)
        pk.msrep_timing_only(None)
        return ev, kt

    # warmup steps are cold too, so that every launch of a kernel in this run
    # is alike (a profiler's per-kernel average then matches the timed one);
    # they time every kernel, to find the dominant one
    _, kt_warm = timed_steps(args.warmup)
    if args.copy_calibration:
        src = torch.empty(COPY_CAL_BYTES, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        scrub.fill_(1)
        dst.copy_(src)
        del src, dst
    torch.cuda.synchronize()
    # the dominant kernel: the largest share of the step's time among the
    # SpMV kernels proper (not the boundary merges)
    dom = None
    if priced_of(kt_warm):
        dom = max(priced_of(kt_warm).items(), key=lambda kv: kv[1][1])[0]
    # ---- timed region: K steps, each SpMV cold and bracketed by events; the
    # library brackets the dominant kernel with HIP events on the same stream
    # (its duration for the roofline)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev, ktime = timed_steps(args.steps, only=dom)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    # ---- after it: the per-kernel breakdown of every format (all kernels
    # timed, so these steps are slower than the timed ones)
    _, kt_all = timed_steps(args.steps)
    torch.cuda.synchronize()
    cold_ms = {f: float(np.mean([a.elapsed_time(b) for a, b in ev[f]])) for f in fmts}
    # ---- warm (optional): back-to-back SpMVs of one format
    warm_ms = {}
    for f in fmts if args.warm else []:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            spmv(f)
        e1.record()
        torch.cuda.synchronize()
        warm_ms[f] = e0.elapsed_time(e1) / args.steps
    # ---- correctness of this run's results: every format against the FP64
    # oracle (Dot2) on the original values; for FP32 / BF16 values also
    # against the oracle on the stored values (the accumulation error alone)
    errs = {}
    if not args.no_check:
        if ref is None:
            ref = oracle.spmv_csr(A.m, A.n, A.ptr, A.col, A.val, x64)
        y_ref, sc = ref
        ref_st = None
        if vt != pk.F64:
            ref_st = oracle.spmv_csr(A.m, A.n, A.ptr, A.col, stored_as_f64(stored_values(A.val, vt), vt),
                                     x64.astype(np.float32).astype(np.float64))
        for f in fmts:
            yg = ys[f].double().cpu().numpy()
            e = {"max_scaled_error_vs_fp64_oracle":
                 float(np.max(np.abs(yg - y_ref) / np.where(sc > 0, sc, 1.0)))}
            if ref_st is not None:
                e["max_scaled_error_vs_oracle_on_stored_values"] = float(
                    np.max(np.abs(yg - ref_st[0]) / np.where(ref_st[1] > 0, ref_st[1], 1.0)))
            errs[f] = e
    step_ms = sum(cold_ms.values())
    flops = 2.0 * A.nnz * len(fmts)
    per_fmt = {}
    for f in fmts:
        b = fmt_bytes(f)
        each = sorted(a.elapsed_time(b_) for a, b_ in ev[f])
        per_fmt[f] = {"ms_cold": round(cold_ms[f], 4),
                      "ms_cold_median": round(float(np.median(each)), 4),
                      "ms_cold_min": round(each[0], 4),
                      "gflops_cold": round(2.0 * A.nnz / cold_ms[f] / 1e6, 2),
                      "gbs_cold": round(b / cold_ms[f] / 1e6, 1),
                      "frac_cold": round(b / cold_ms[f] / 1e6 / HBM_PEAK_GBS, 4),
                      "alg_bytes": int(b), "partition_ms": round(part_ms[f], 4),
                      "prepare_ms": round(prep_ms[f], 4),
                      "entry": "msrep_spmv" if args.unprepared else "msrep_spmv_prepared",
                      "np": parts[f].np,
                      "tune": {"k_per_lane": tunes[f].k_per_lane or 4,
                               "waves_per_wg": tunes[f].waves_per_wg or 4,
                               "nnz_per_wave": tunes[f].nnz_per_wave,
                               "pipeline": tunes[f].pipeline or 2,
                               "resident": tunes[f].resident}}
        if f in warm_ms:
            per_fmt[f]["ms_warm"] = round(warm_ms[f], 4)
            per_fmt[f]["gbs_warm"] = round(b / warm_ms[f] / 1e6, 1)
        per_fmt[f]["kernels_us"] = {k: round(t / c * 1e3, 2) for (g, k), (c, t) in kt_all.items()
                                    if g == f}
        per_fmt[f].update(errs.get(f, {}))
    priced = priced_of(ktime)
    if not priced:  # no warmup: take the dominant kernel from the breakdown
        priced = priced_of(kt_all)
    (dom_f, kname), (kc, kt) = max(priced.items(), key=lambda kv: kv[1][1])
    k_ms = kt / kc
    k_bytes = fmt_bytes(dom_f)
    achieved = k_bytes / (k_ms * 1e-3) / 1e9
    traffic = load_traffic("%s/%s/%s" % (kname, wl["workload"], vname))
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "kernel": kname, "format": dom_f,
            "kernel_avg_us": round(k_ms * 1e3, 2), "alg_bytes_per_launch": int(k_bytes),
            "alg_bytes_basis": "the %s SpMV's own bytes (values, indices, pointer, x and y, "
                               "each moved once), whichever kernel of the format moves them"
                               % dom_f,
            "path": {"format": dom_f, "ms": round(cold_ms[dom_f], 4),
                     "achieved": round(k_bytes / cold_ms[dom_f] / 1e6, 1),
                     "frac": round(k_bytes / cold_ms[dom_f] / 1e6 / HBM_PEAK_GBS, 4)}}
    out = {"step_ms": step_ms, "gflops": flops / (step_ms * 1e-3) / 1e9,
           "config": dict(wl, formats=fmts, value_type=vname, split=args.split),
           "roofline": roof, "per_format": per_fmt, "wall_s_timed_region": round(wall, 3),
           "ref": ref}
    if args.overheads:
        out["overheads"] = overheads(args, mats, part_ms, prep_ms, cold_ms, kt_all)
    del mats, ws, scrub, ys, x
    torch.cuda.empty_cache()
    return out


# kernels whose launch is priced against the SpMV's algorithmic bytes (the
# per-format SpMV kernels proper; the boundary merges and the structure-only
# CSC kernels are not)
PRICED_KERNELS = ("spmv_csr_seg", "spmv_coo_seg", "csc_scatter", "csc_reduce", "cscw_tile", "cscw_merge")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="stencil256",
                    choices=["rmat20", "stencil256", "uniform4096", "batched", "serve"])
    ap.add_argument("--rhs", type=int, default=0,
                    help="k > 0: time msrep_spmm with k right-hand sides (CSR) instead")
    ap.add_argument("--count", type=int, default=512, help="batched / serving pool size")
    ap.add_argument("--requests", type=int, default=10000,
                    help="serving: requests per load point (the plain path serves a quarter)")
    ap.add_argument("--rates", default="0.1,0.5,0.9,1.2", help="serving: fractions of capacity")
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--steps-per-tick", type=int, default=0,
                    help="serving: most steps of one request per tick (0: library default)")
    ap.add_argument("--vtype", default="f64", choices=["f64", "f32", "bf16"])
    ap.add_argument("--formats", default="csr,csc,coo")
    ap.add_argument("--nnz-per-wave", type=int, default=0, help="partition size (0: tuned)")
    ap.add_argument("--k", type=int, default=0)
    ap.add_argument("--wpb", type=int, default=0)
    ap.add_argument("--pipeline", type=int, default=0)
    ap.add_argument("--resident", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle checks")
    ap.add_argument("--only", action="store_true",
                    help="the named workload alone (no R-MAT or precision blocks)")
    ap.add_argument("--autotune", action="store_true", help="tune every format first")
    ap.add_argument("--overheads", action="store_true",
                    help="also time conversion, partition build and merge against the SpMV")
    ap.add_argument("--split", default="nnz", choices=["nnz", "rows"],
                    help="rows: the paper's equal-rows baseline partitions (same np)")
    ap.add_argument("--unprepared", action="store_true",
                    help="time msrep_spmv (structure work in every call) instead of "
                         "msrep_spmv_prepare once + msrep_spmv_prepared")
    ap.add_argument("--warm", action="store_true",
                    help="also time back-to-back (cache-warm) SpMVs of each format")
    ap.add_argument("--ceiling", action="store_true",
                    help="also measure the plain-stream HBM ceiling with --only")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB copy (counter calibration)")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "KERNEL", "KEY"))
    ap.add_argument("--trace-summary", nargs=2, metavar=("TRACE_DIR", "OUT_NAME"))
    ap.add_argument("--counter-summary", nargs="+", metavar="ARG",
                    help="OUT_NAME KERNELS(comma-separated) PMC_DIR...: counter means per kernel")
    ap.add_argument("--command", default="", help="command line recorded in a summary")
    ap.add_argument("--bench-json", default=None, help="the traced run's output (trace summary)")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary, command=args.command)
        return 0
    if args.trace_summary:
        trace_summary(*args.trace_summary, command=args.command, bench_json=args.bench_json)
        return 0
    if args.counter_summary:
        out_name, kernels, *dirs = args.counter_summary
        counter_summary(dirs, out_name, kernels.split(","), command=args.command)
        return 0
    if args.gpus != 1:
        print("bench.py: one GPU only; --gpus %d is not supported (how the path would "
              "shard across GPUs is a design note, not code)" % args.gpus, file=sys.stderr)
        return 2

    import torch

    import paper_2209_07552_amd as pk

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    vt = {"f64": pk.F64, "f32": pk.F32, "bf16": pk.BF16}[args.vtype]
    if args.rhs > 0:
        return bench_spmm(args, vt)
    if args.workload == "batched":
        return bench_batched(args, vt)
    if args.workload == "serve":
        return bench_serve(args, vt)
    fmts = [f for f in args.formats.split(",") if f]
    A, x64, wl = gen_workload(args.workload)
    r = measure_matrix(args, A, x64, wl, args.workload, vt, fmts)
    out = {
        "metric": "SpMV GFLOP/s (cold HBM; CSR+CSC+COO per step)",
        "value": round(r["gflops"], 3),
        "unit": "GFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(r["step_ms"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.vtype, "data": "synthetic",
        "config": r["config"],
        "roofline": r["roofline"],
        "per_format": r["per_format"],
        "wall_s_timed_region": r["wall_s_timed_region"],
    }
    if "overheads" in r:
        out["overheads"] = r["overheads"]
    errs = [v["max_scaled_error_vs_fp64_oracle"] for v in r["per_format"].values()
            if "max_scaled_error_vs_fp64_oracle" in v]
    if errs:
        key = "max_scaled_error_vs_oracle" if vt == pk.F64 else "max_scaled_error_vs_fp64_oracle"
        out[key] = max(errs)
    if not args.only and args.workload == "stencil256" and vt == pk.F64:
        # pattern (1), precision: the same stencil with FP32 and BF16 stored
        # values (FP32 x, y and accumulation), same launch shapes
        prec = {}
        for pv in (pk.F32, pk.BF16):
            rp = measure_matrix(args, A, x64, wl, args.workload, pv, fmts, ref=r["ref"])
            prec[pk._abi.VT_NAMES[pv]] = {
                "ms_per_step": round(rp["step_ms"], 4), "gflops": round(rp["gflops"], 3),
                "speedup_vs_f64": round(r["step_ms"] / rp["step_ms"], 3),
                "roofline": rp["roofline"], "per_format": rp["per_format"]}
        out["precision"] = prec
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(A, x64)
    if not args.only or args.ceiling:
        # what plain streams reach here, beside the roofline's 8 TB/s peak
        ceil = stream_ceiling()
        out["stream_ceiling"] = ceil
        if out["roofline"].get("unit") == "GB/s":
            out["roofline"]["frac_of_stream_read"] = round(
                out["roofline"]["achieved"] / ceil["read_gbs"], 4)
    if not args.only and args.workload == "stencil256" and vt == pk.F64:
        # the power-law matrix: the same step on R-MAT scale 20
        del A, x64
        B, xb, wlb = gen_workload("rmat20")
        rb = measure_matrix(args, B, xb, wlb, "rmat20", vt, fmts)
        out["rmat20"] = {"config": rb["config"], "ms_per_step": round(rb["step_ms"], 4),
                         "gflops": round(rb["gflops"], 3), "roofline": rb["roofline"],
                         "per_format": rb["per_format"]}
    print(json.dumps(out), flush=True)
    return 0


def stream_ceiling(reps=5):
    """The HBM rate plain streams reach on this GPU (msrep_probe_stream):
    one pass of 16-byte loads over 2 GiB, and a 2 GiB copy, each cold
    (scrubbed before), median of reps.  The practical ceiling beside the
    8 TB/s peak for kernels that stream their operands."""
    import torch

    import paper_2209_07552_amd as pk
    dev = torch.device("cuda:0")
    nbytes = 2 << 30
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty(nbytes // 8, dtype=torch.float64, device=dev)
    scrub = torch.empty(SCRUB_BYTES, dtype=torch.uint8, device=dev)
    out = {"bytes": nbytes, "kind": "msrep_probe_stream"}
    for mode, key, mult in ((0, "read_gbs", 1), (1, "copy_gbs", 2)):
        best = None
        for blocks in (2048, 65536):
            ts = []
            for _ in range(reps):
                scrub.fill_(1)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                pk.msrep_probe_stream(src, dst, mode, blocks)
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            ms = float(np.median(ts))
            if best is None or ms < best[0]:
                best = (ms, blocks)
        out[key] = round(mult * nbytes / best[0] / 1e6, 1)
        out[key.replace("_gbs", "_blocks")] = best[1]
    out["copy_counts"] = "read + write bytes"
    del src, dst, scrub
    torch.cuda.empty_cache()
    return out


def _timed(fn, reps):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_spmm(args, vt):
    """Y = A*X for k right-hand sides (msrep_spmm, CSR) on the R-MAT or
    stencil workload, each call cold in HBM, against k single-vector CSR
    SpMVs (msrep_spmv, the tuned launch shape) over the same columns after
    one scrub.  The roofline is that of the spmm_csr kernel: A, its row
    pointer, X and Y each moved once per pass of up to eight columns."""
    import torch

    import oracle
    import paper_2209_07552_amd as pk
    import synth
    dev = torch.device("cuda:0")
    k = args.rhs
    t0 = time.time()
    if args.workload == "stencil256":
        A, _ = synth.stencil7_csr(256, seed=0)
        wl = {"workload": "laplace3d-7pt-256^3", "rows": A.m, "cols": A.n, "nnz": A.nnz}
    else:
        A, _ = synth.rmat_csr(scale=20, edge_factor=16, seed=0)
        wl = {"workload": "rmat-scale20-ef16", "rows": A.m, "cols": A.n, "nnz": A.nnz,
              "abcd": [0.57, 0.19, 0.19, 0.05]}
    log("generated %s in %.1fs" % (wl["workload"], time.time() - t0))
    vdt = np.float64 if vt == pk.F64 else np.float32
    tdt = torch.float64 if vt == pk.F64 else torch.float32
    vb, xb = pk._abi.VALUE_BYTES[vt], (8 if vt == pk.F64 else 4)
    sv = A.val.astype(vdt) if vt != pk.BF16 else synth.bf16_bits(A.val.astype(np.float32))
    M = pk.Mat(pk.CSR, vt, A.m, A.n, ptr=A.ptr, idx=A.col, val=sv)
    npw = args.nnz_per_wave or {"stencil256": 2048}.get(args.workload, 512)
    P = pk.msrep_build_partition(M, max(1, -(-A.nnz // npw)))
    rng = np.random.default_rng(1)
    X64 = rng.uniform(-1, 1, (A.n, k))
    Xd = torch.from_numpy(X64.astype(vdt)).to(dev)
    Yd = torch.zeros((A.m, k), dtype=tdt, device=dev)
    ws = torch.zeros(max(256, pk.msrep_spmm_ws_bytes(M, P.np, k)), dtype=torch.uint8, device=dev)
    scrub = torch.empty(SCRUB_BYTES, dtype=torch.uint8, device=dev)

    def spmm():
        pk.msrep_spmm(M, P, Xd, Yd, 1.0, 0.0, ws=ws)

    def steps(n_, timing):
        evs, kt = [], (0, 0.0)
        for _ in range(n_):
            scrub.fill_(1)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            pk.msrep_timing(timing)
            pk.msrep_timing_only("spmm_csr" if timing else None)
            e0.record()
            spmm()
            e1.record()
            if timing:
                for name, (c, t) in pk.msrep_timing_read().items():
                    if name == "spmm_csr":
                        kt = (kt[0] + c, kt[1] + t)
            evs.append((e0, e1))
        pk.msrep_timing(False)
        pk.msrep_timing_only(None)
        torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in evs], kt

    steps(args.warmup, False)
    if args.copy_calibration:  # a plain copy of known size for the byte counters
        src = torch.empty(COPY_CAL_BYTES, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        scrub.fill_(1)
        dst.copy_(src)
        del src, dst
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ms, kt = steps(args.steps, True)
    wall = time.perf_counter() - wall0
    ms_spmm = float(np.mean(ms))
    passes = []
    left = k
    while left > 0:
        nr = 8 if left >= 8 else 4 if left >= 4 else 2 if left >= 2 else 1
        passes.append(nr)
        left -= nr
    k_us = kt[1] / kt[0] * 1e3 if kt[0] else None  # per pass launch (None: k = 1 ran the SpMV kernel)
    pass_bytes = [A.nnz * (vb + 4) + (A.m + 1) * 4 + nr * (A.n + A.m) * xb for nr in passes]
    k_bytes = float(np.mean(pass_bytes))
    achieved = k_bytes / (k_us * 1e-6) / 1e9 if k_us else None
    call_bytes = sum(pass_bytes)
    # comparator: k single-vector SpMVs (tuned CSR launch shape and partitions).
    # Skipped in counter runs (--copy-calibration): its column copies are
    # copy kernels too and would blur the calibration copy's readings.
    if args.copy_calibration:
        print(json.dumps({"metric": "SpMM counter run", "ms_per_step": round(ms_spmm, 4)}), flush=True)
        return 0
    st = DEFAULT_TUNES.get(args.workload, {}).get("csr", (512, 4, 8, 2, 1))
    tune = pk.Tune(k_per_lane=st[1], waves_per_wg=st[2], nnz_per_wave=st[0], pipeline=st[3],
                   resident=st[4])
    P1 = pk.msrep_build_partition(M, max(1, -(-A.nnz // st[0])))
    ws1 = torch.zeros(max(256, pk.msrep_spmv_ws_bytes(M, P1.np)), dtype=torch.uint8, device=dev)
    xs = [Xd[:, j].contiguous() for j in range(k)]
    ys = [torch.zeros(A.m, dtype=tdt, device=dev) for _ in range(k)]

    def spmvs():
        for j in range(k):
            pk.msrep_spmv(M, P1, xs[j], ys[j], 1.0, 0.0, tune, ws=ws1)
    ms_v = []
    for i in range(args.warmup + args.steps):
        scrub.fill_(1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        spmvs()
        e1.record()
        torch.cuda.synchronize()
        if i >= args.warmup:
            ms_v.append(e0.elapsed_time(e1))
    ms_spmv = float(np.mean(ms_v))
    flops = 2.0 * A.nnz * k
    out = {"metric": "SpMM GFLOP/s (k right-hand sides, CSR, cold HBM)",
           "value": round(flops / (ms_spmm * 1e-3) / 1e9, 3), "unit": "GFLOP/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_spmm, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": args.vtype, "data": "synthetic",
           "config": dict(wl, rhs=k, layout="row-major X (n x k), Y (m x k)", np=P.np,
                          nnz_per_wave=npw, passes=passes),
           "alg_gbs": round(call_bytes / (ms_spmm * 1e-3) / 1e9, 1),
           "roofline": None if k_us is None else {
               "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
               "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
               "traffic": load_traffic("spmm_csr/%s/%s/k%d" % (wl["workload"], args.vtype, k)),
               "kernel": "spmm_csr", "kernel_avg_us": round(k_us, 2),
               "alg_bytes_per_launch": int(k_bytes)},
           "k_spmv": {"ms": round(ms_spmv, 4), "gflops": round(flops / (ms_spmv * 1e-3) / 1e9, 3),
                      "entry": "msrep_spmv x %d" % k, "np": P1.np},
           "speedup_vs_k_spmv": round(ms_spmv / ms_spmm, 3),
           "wall_s_timed_region": round(wall, 3)}
    # correctness of this run's Y against the oracle, and the oracle's own
    # rate (its whole product, one thread) as the CPU baseline
    if not args.no_cpu and vt == pk.F64:
        c0 = time.perf_counter()
        ref, sc = oracle.spmm_csr(A.m, A.n, A.ptr, A.col, A.val, X64)
        cpu_s = time.perf_counter() - c0
        yg = Yd.double().cpu().numpy()
        err = float(np.max(np.abs(yg - ref) / np.where(sc > 0, sc, 1.0)))
        out["cpu_baseline"] = {"value": round(flops / cpu_s / 1e9, 4), "unit": "GFLOP/s",
                               "cores": 1, "kind": "oracle",
                               "sample": "one whole product (%d columns), FP64 Dot2" % k}
        out["max_scaled_error_vs_oracle"] = err
    print(json.dumps(out), flush=True)
    return 0


def bench_batched(args, vt):
    """512 uneven matrices (log-uniform rows in [1e3, 2e5], half uniform 4-64
    nnz/row, half R-MAT-like) in one persistent hipGraph launch, against the
    plain path (one msrep_spmv launch per matrix, same partitions).  Every
    matrix's y of the batched run is then checked against the FP64 oracle."""
    import torch

    import oracle
    import paper_2209_07552_amd as pk
    import synth
    dev = torch.device("cuda:0")
    t0 = time.time()
    mats = synth.batched_set(args.count, seed=0)
    log("generated %d matrices in %.1fs" % (args.count, time.time() - t0))
    vdt = np.float64 if vt == pk.F64 else np.float32
    Ms = [pk.Mat(pk.CSR, vt, A.m, A.n, ptr=A.ptr, idx=A.col, val=A.val.astype(vdt)) for A, _ in mats]
    xs = [torch.from_numpy(x.astype(vdt)).to(dev) for _, x in mats]
    ys = [torch.zeros(A.m, dtype=xs[0].dtype, device=dev) for A, _ in mats]
    nnz = sum(A.nnz for A, _ in mats)
    xb = 8 if vt == pk.F64 else 4
    byts = sum(A.nnz * (pk._abi.VALUE_BYTES[vt] + 4) + (A.m + 1) * 4 + (A.n + A.m) * xb for A, _ in mats)
    # autotuned partition size per matrix class (uniform / power-law x size)
    t0 = time.time()
    classes = {}
    for k, (A, _) in enumerate(mats):
        key = (k % 2, int(np.log10(max(A.m, 10))))
        classes.setdefault(key, k)
    tuned = ({} if args.nnz_per_wave else
             {key: pk.msrep_autotune(Ms[k], xs[k]) for key, k in classes.items()})
    def class_tune(k, A):
        return tuned[(k % 2, int(np.log10(max(A.m, 10))))]

    def plan_tunes(floor):
        return [pk.Tune(k_per_lane=args.k or 4, waves_per_wg=args.wpb or 4,
                        nnz_per_wave=(args.nnz_per_wave or
                                      max(class_tune(k, A).nnz_per_wave, floor)),
                        pipeline=args.pipeline)
                for k, (A, _) in enumerate(mats)]
    log("autotuned %d classes in %.1fs" % (len(classes), time.time() - t0))
    # the persistent kernel pays a fixed latency per work item (its chain of
    # descriptor and partition loads), so the plan's items may want more
    # nonzeros than the single-matrix tuner's partitions: time the plan with
    # the tuned sizes and with floors of 2048-8192 nonzeros, keep the fastest
    floors = [0] if args.nnz_per_wave else [0, 2048, 4096, 8192]
    best = None
    for floor in floors:
        tn = plan_tunes(floor)
        pl = pk.msrep_plan_create(Ms, tn)
        for _ in range(2):
            pk.msrep_spmv_batched(pl, xs, ys)
        t = _timed(lambda: pk.msrep_spmv_batched(pl, xs, ys), 3)
        log("plan item floor %d: %.3f ms (%d items)" % (floor, t, pl.items()))
        if best is None or t < best[0]:
            best = (t, floor, tn)
        pl.destroy()
    _, floor, tunes = best
    plan = pk.msrep_plan_create(Ms, tunes)
    for _ in range(args.warmup):
        pk.msrep_spmv_batched(plan, xs, ys)
    ms_b = _timed(lambda: pk.msrep_spmv_batched(plan, xs, ys), args.steps)
    yb = [y.double().cpu().numpy() for y in ys]
    # plain path: one launch (plus merge) per matrix, each with its class's
    # tuned launch shape and partition size
    ptunes = ([pk.Tune(k_per_lane=args.k or 4, waves_per_wg=args.wpb or 4,
                       nnz_per_wave=args.nnz_per_wave, pipeline=args.pipeline)] * len(mats)
              if args.nnz_per_wave else [class_tune(k, A) for k, (A, _) in enumerate(mats)])
    parts = [pk.msrep_build_partition(M, max(1, -(-M.nnz // t.nnz_per_wave)))
             for M, t in zip(Ms, ptunes)]
    ws = torch.zeros(1 << 26, dtype=torch.uint8, device=dev)

    def plain():
        for M, P, x, y, t in zip(Ms, parts, xs, ys, ptunes):
            pk.msrep_spmv(M, P, x, y, 1.0, 0.0, t, ws=ws)
    for _ in range(args.warmup):
        plain()
    ms_p = _timed(plain, max(1, args.steps // 4))
    # every matrix's batched result against the FP64 oracle on the original
    # (FP64) values; for FP32 values also against the oracle on the stored
    # values and FP32-rounded x
    err, err_st = 0.0, 0.0
    if not args.no_check:
        for (A, x), yg in zip(mats, yb):
            ref, sc = oracle.spmv_csr(A.m, A.n, A.ptr, A.col, A.val, x)
            err = max(err, float(np.max(np.abs(yg - ref) / np.where(sc > 0, sc, 1.0))))
            if vt != pk.F64:
                r2, s2 = oracle.spmv_csr(A.m, A.n, A.ptr, A.col,
                                         A.val.astype(np.float32).astype(np.float64),
                                         x.astype(np.float32).astype(np.float64))
                err_st = max(err_st, float(np.max(np.abs(yg - r2) / np.where(s2 > 0, s2, 1.0))))
    out = {"metric": "batched SpMV/s (%d uneven matrices, one persistent hipGraph launch)" % args.count,
           "value": round(args.count / (ms_b * 1e-3), 1), "unit": "SpMV/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_b, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.vtype,
           "data": "synthetic",
           "config": {"workload": "batched-%d" % args.count, "total_nnz": nnz, "items": plan.items(),
                      "item_floor_nnz": floor},
           "gflops": round(2.0 * nnz / (ms_b * 1e-3) / 1e9, 2),
           "alg_gbs": round(byts / (ms_b * 1e-3) / 1e9, 1),
           "frac": round(byts / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "plain_path": {"ms_per_batch": round(ms_p, 4),
                          "spmv_per_s": round(args.count / (ms_p * 1e-3), 1)},
           "speedup_vs_plain": round(ms_p / ms_b, 3)}
    if not args.no_check:
        out["max_scaled_error_vs_fp64_oracle"] = err
        out["checked"] = "all %d matrices, every row" % args.count
        if vt != pk.F64:
            out["max_scaled_error_vs_oracle_on_stored_values"] = err_st
    print(json.dumps(out), flush=True)
    return 0


def plain_serve(pool, trace, vt, seed=0, nnz_per_wave=1024):
    """The plain path on a serving trace: every pool matrix resident with its
    partitions, requests served one at a time in arrival order (a request
    waits for its arrival and for the one before it), each step one device x
    generation (the server's generator) and one msrep_spmv launch.  Latency
    = arrival to the completion of the request's last step, on the same
    trace clock as the server's.  Returns the latencies in ms."""
    import torch

    import paper_2209_07552_amd as pk
    from paper_2209_07552_amd import serving
    dev = torch.device("cuda:0")
    vdt = np.float64 if vt == pk.F64 else np.float32
    used = sorted({q.matrix for q in trace})
    Ms, Ps = {}, {}
    for k in used:
        A = pool[k]
        Ms[k] = pk.Mat(pk.CSR, vt, A.m, A.n, ptr=A.ptr, idx=A.col, val=A.val.astype(vdt))
        Ps[k] = pk.msrep_build_partition(Ms[k], max(1, -(-A.nnz // nnz_per_wave)))
    mmax = max(pool[k].m for k in used)
    nmax = max(pool[k].n for k in used)
    ydt = pk._abi.vector_dtype(vt)
    xbuf = torch.empty(nmax, dtype=ydt, device=dev)
    ybuf = torch.empty(mmax, dtype=ydt, device=dev)
    ws = torch.zeros(1 << 26, dtype=torch.uint8, device=dev)
    done = torch.cuda.Event()
    torch.cuda.synchronize()
    order = sorted(range(len(trace)), key=lambda i: trace[i].t_arrive)
    lat = [0.0] * len(trace)
    t0 = time.perf_counter()
    for i in order:
        q = trace[i]
        A = pool[q.matrix]
        while time.perf_counter() - t0 < q.t_arrive:
            pass
        x, y = xbuf[:A.n], ybuf[:A.m]
        for j in range(q.steps):
            serving.fill_x(x, seed, q.rid, j)
            pk.msrep_spmv(Ms[q.matrix], Ps[q.matrix], x, y, ws=ws)
        done.record()
        done.synchronize()
        lat[i] = (time.perf_counter() - t0 - q.t_arrive) * 1e3
    return lat


def bench_serve(args, vt):
    """Poisson request stream over a pool of batched-style matrices; each
    request = one matrix + 10..100 SpMVs with fresh x; arena budget as given.
    Rates are fractions of the measured batched capacity.  Beside it, the
    plain path on the same traces: one request at a time, one msrep_spmv
    launch per SpMV, x generated on the device.  A sample of served results
    is checked against the FP64 oracle."""
    import oracle
    import paper_2209_07552_amd as pk
    from paper_2209_07552_amd import serving
    import synth
    t0 = time.time()
    pool = [A for A, _ in synth.batched_set(args.count, seed=0)]
    log("generated pool of %d in %.1fs" % (len(pool), time.time() - t0))
    budget = int(args.budget_gb * (1 << 30))
    mean_steps = 55.0
    # capacity estimate from a saturated run: SpMVs per second of the mix,
    # with enough requests (four per pool matrix) that the run is mostly
    # steady state rather than first uploads and a draining tail
    probe = synth.serving_trace(max(64, 4 * args.count), rate=1e9, pool=len(pool), seed=99)
    spt = args.steps_per_tick
    npw = args.nnz_per_wave or 1024  # the server's partition size (nonzeros per wavefront)
    _, st = serving.serve(pool, probe, budget_bytes=budget, vtype=vt, max_slots=256,
                          nnz_per_wave=npw, steps_per_tick=spt)
    cap_req = st["spmv_per_s"] / mean_steps
    log("saturated mix: %.0f SpMV/s -> capacity ~%.1f req/s" % (st["spmv_per_s"], cap_req))
    points = []
    n_plain = max(1, args.requests // 4)
    for f in [float(v) for v in args.rates.split(",")]:
        trace = synth.serving_trace(args.requests, rate=max(f * cap_req, 1e-3), pool=len(pool), seed=1)
        _, st = serving.serve(pool, trace, budget_bytes=budget, vtype=vt, max_slots=256,
                              nnz_per_wave=npw, steps_per_tick=spt)
        pt = {"load": f, "rate_req_s": round(f * cap_req, 2),
              "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
              "req_per_s": round(st["req_per_s"], 2),
              "spmv_per_s": round(st["spmv_per_s"], 1), "gflops": round(st["gflops"], 2),
              "peak_active": st["peak_active"], "ticks": st["ticks"]}
        if f <= 1.0:  # the plain path on the first requests of the same trace
            lat = plain_serve(pool, trace[:n_plain], vt)
            pt["plain"] = {"requests": n_plain,
                           "p50_ms": round(float(np.percentile(lat, 50)), 3),
                           "p99_ms": round(float(np.percentile(lat, 99)), 3)}
        points.append(pt)
        log(json.dumps(pt))
    # accuracy of served results: a separate run that keeps the last y of a
    # sample of requests, each checked against the FP64 oracle on its matrix
    # and that step's x (for FP32 pools also on the stored values)
    chk = synth.serving_trace(64, rate=0.5 * cap_req, pool=len(pool), seed=2)
    res, _ = serving.serve(pool, chk, budget_bytes=budget, vtype=vt, max_slots=256,
                           nnz_per_wave=npw, keep_y=range(0, 64, 4), steps_per_tick=spt)
    err = err_st = 0.0
    for i in range(0, 64, 4):
        q, A = chk[i], pool[chk[i].matrix]
        x = synth.serving_x(A.n, 0, q.rid, q.steps - 1)
        ref, sc = oracle.spmv_csr(A.m, A.n, A.ptr, A.col, A.val, x)
        yg = np.asarray(res[i].y, np.float64)
        err = max(err, float(np.max(np.abs(yg - ref) / np.where(sc > 0, sc, 1.0))))
        if vt != pk.F64:
            r2, s2 = oracle.spmv_csr(A.m, A.n, A.ptr, A.col, A.val.astype(np.float32).astype(np.float64),
                                     x.astype(np.float32).astype(np.float64))
            err_st = max(err_st, float(np.max(np.abs(yg - r2) / np.where(s2 > 0, s2, 1.0))))
    best = max(points, key=lambda p: p["req_per_s"])
    out = {"metric": "served p50/p99 latency and req/s (Poisson, continuous batching)",
           "value": best["req_per_s"], "unit": "req/s", "n_gpus": 1, "steps": args.requests,
           "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": args.vtype, "data": "synthetic",
           "config": {"workload": "serve-pool%d" % len(pool), "budget_gb": args.budget_gb,
                      "steps_per_request": "U{10..100}",
                      "steps_per_tick": spt or "by load, up to 64", "nnz_per_wave": npw},
           "points": points,
           "plain_path": "the same trace's first %d requests, one at a time in arrival order "
                         "(queueing included), x generated on the device, one msrep_spmv per "
                         "step, matrices and partitions resident" % n_plain,
           "max_scaled_error_vs_fp64_oracle": err,
           "checked": "last y of 16 of 64 requests served at 0.5x capacity, every row"}
    if vt != pk.F64:
        out["max_scaled_error_vs_oracle_on_stored_values"] = err_st
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
