#!/usr/bin/env python3
"""Benchmark of the equal-nnz partitioned SpMV (msRep, arXiv 2209.07552) on
one MI355X.

Default workload: the power-law FP64 configuration -- an R-MAT scale-20
matrix (1,048,576 rows and columns, edge factor 16, a/b/c/d =
.57/.19/.19/.05, duplicates merged; values and x ~ U(-1, 1), seed 0) stored
as CSR, CSC and COO, each split into equal-nnz partitions over the CUs.  One
step is y = A*x in each of the three formats (partitions and matrices
resident in HBM, boundary merges included).  Every SpMV of the timed region
runs cache-cold: a 512 MiB scrub write between SpMVs evicts the 256 MB
Infinity Cache, and HIP events on the library's stream bracket each SpMV, so
the reported throughput is the SpMV time alone.  A warm (back-to-back) figure
is reported beside it.

Prints one JSON line (rank 0, N = 1).  --gpus N > 1 exits: this build runs on
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
               "coo_any": (1024, 4, 2, 1, 0)},
    "stencil256": {"csr": (2048, 4, 4, 2, 0), "coo": (1024, 4, 2, 2, 0),
                   "csc": (1024, 4, 2, 2, 0), "coo_any": (1024, 4, 2, 2, 0)},
}
SCRUB_BYTES = 512 << 20


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_formats(A, any_order=False):
    """CSC and row-sorted COO arrays of a CSR matrix (plain numpy input
    preparation: stable sort by column), and with any_order the COO in a
    seeded random order."""
    rows = np.repeat(np.arange(A.m, dtype=np.int32), np.diff(A.ptr))
    perm = np.argsort(A.col, kind="stable")
    cptr = np.zeros(A.n + 1, np.int64)
    np.cumsum(np.bincount(A.col, minlength=A.n), out=cptr[1:])
    out = {"csr": (A.ptr, A.col, A.val),
           "csc": (cptr.astype(np.int32), rows[perm], A.val[perm]),
           "coo": (rows, A.col, A.val)}
    if any_order:  # COO in a seeded random order
        shuf = np.random.default_rng(0).permutation(A.nnz)
        out["coo_any"] = (rows[shuf], A.col[shuf], A.val[shuf])
    return out


def equal_rows_partition(M, H, fmt, np_, dev):
    """The paper's baseline split (equal rows, or equal columns for CSC,
    unequal nonzeros) as partition records the SpMV kernels take: partition
    i starts at major index floor(i*rows/np); its fields follow the same
    definitions as the equal-nnz build (row containing start_idx and end_idx,
    local pointer clamped to the partition, start_row + 2i offsets), and its
    flags are 0 since it never splits a row.  Host numpy, for comparison
    runs only."""
    import torch
    import paper_2209_07552_amd as pk
    a, b, _ = H[fmt]
    rows = M.major
    nnz = int(M.nnz)
    bnd = (np.arange(np_ + 1, dtype=np.int64) * rows) // np_
    if fmt == "coo":
        first = np.searchsorted(np.asarray(a, np.int64), bnd, "left").astype(np.int64)
        ptr = None
    else:
        ptr = np.asarray(a, np.int64)
        first = ptr[bnd]
    rec = np.zeros(np_, pk.PART_DTYPE)
    s0, e0 = first[:-1], first[1:] - 1
    rec["start_idx"], rec["end_idx"] = s0, e0
    if fmt == "coo":
        ri = np.asarray(a, np.int64)
        srow = np.where(s0 < nnz, ri[np.minimum(s0, nnz - 1)], rows) if nnz else np.full(np_, rows)
        erow = np.where(e0 >= s0, ri[np.maximum(e0, 0)] if nnz else 0, srow - 1)
    else:
        def bs(k):  # the row containing nonzero k: max r with ptr[r] <= k
            return np.searchsorted(ptr, k, "right") - 1
        srow = np.where(s0 < nnz, bs(s0), rows)
        erow = np.where(e0 >= s0, bs(np.maximum(e0, 0)), srow - 1)
    rec["start_row"], rec["end_row"] = srow, erow
    rec["lptr_off"] = srow + 2 * np.arange(np_, dtype=np.int64)
    parts = torch.from_numpy(rec.view(np.uint8).copy()).to(dev)
    if fmt == "coo":
        return pk.Partition(M, np_, parts, None, torch.zeros(1, dtype=torch.int64, device=dev))
    cap = rows + 2 * np_
    lp = np.zeros(cap, np.int32)
    for i in range(np_):
        R = int(erow[i] - srow[i] + 1)
        if R <= 0:
            lp[rec["lptr_off"][i]] = 0
            continue
        seg = ptr[srow[i]:srow[i] + R + 1]
        lp[rec["lptr_off"][i]:rec["lptr_off"][i] + R + 1] = np.clip(seg, s0[i], e0[i] + 1) - s0[i]
    ln = torch.tensor([cap], dtype=torch.int64, device=dev)
    return pk.Partition(M, np_, parts, torch.from_numpy(lp).to(dev), ln)


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


def kernel_alg_bytes(kernel, m, n, nnz, np_, vbytes, xbytes, fmt="csc"):
    """Algorithmic bytes of one launch of a kernel of the SpMV path (one
    launch covers the whole matrix): what its job must read and write, each
    array once.  Bucketed products are FP64 for FP64 values and FP32
    otherwise, each with a 16-bit row offset; for COO in any order the
    scatter reads a column index per nonzero instead of the column pointer."""
    pbytes = 8 if xbytes == 8 else 4
    cols = nnz * 4 if fmt == "coo_any" else (n + 1) * 4
    return {
        "spmv_csr_seg": alg_bytes("csr", m, n, nnz, vbytes, xbytes),
        "spmv_coo_seg": alg_bytes("coo", m, n, nnz, vbytes, xbytes),
        "merge_rows": np_ * (40 + 16),
        "csc_count": nnz * 4,
        "csc_scatter": nnz * (vbytes + 4) + cols + n * xbytes + nnz * (pbytes + 2),
        "csc_reduce": nnz * (pbytes + 2) + m * xbytes,
    }.get(kernel)


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
        cv = [v for (k, n), vs in c.items() if n == ctr and "copy" in k.lower() for v in vs]
        if not kv or not cv:
            raise SystemExit("no %s readings for %s / the copy kernel in %s" % (ctr, kernel, d))
        scale = COPY_CAL_BYTES / (float(np.median(cv)) * 1024.0)
        out[ctr] = (float(np.median(kv)), float(np.median(cv)), scale)
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
    if bench_json:
        rec = json.loads(open(bench_json).read().strip().splitlines()[-1])
        rf = rec.get("roofline", {})
        lines += ["", "# the traced run's bench line: roofline kernel %s, %.2f us per launch by"
                  " HIP events, %.1f GB/s algorithmic (%.4f of %g)" % (
                      rf.get("kernel"), rf.get("kernel_avg_us", float("nan")),
                      rf.get("achieved", float("nan")), rf.get("frac", float("nan")),
                      rf.get("peak", float("nan")))]
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


def cpu_baseline(A, x, y_gpu, budget_s):
    """The FP64 oracle (Dot2 CSR SpMV, one thread) timed on this host over
    whole SpMVs of the same matrix, repeated for about budget_s seconds; also
    the GPU result's largest error relative to (|A||x|)_i."""
    import oracle
    oracle.build(force=False)
    t0 = time.perf_counter()
    y, s = oracle.spmv_csr(A.m, A.n, A.ptr, A.col, A.val, x)
    one = time.perf_counter() - t0
    reps = max(1, int(budget_s / max(one, 1e-3)) - 1)
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.spmv_csr(A.m, A.n, A.ptr, A.col, A.val, x)
    per = (time.perf_counter() - t0) / reps if reps else one
    err = float(np.max(np.abs(y_gpu - y) / np.where(s > 0, s, 1.0)))
    return {"value": round(2.0 * A.nnz / per / 1e9, 4), "unit": "GFLOP/s", "cores": 1,
            "kind": "oracle",
            "sample": "%d full CSR SpMVs of the same matrix (%d nnz), Dot2 FP64, 1 thread"
                      % (reps + 1, A.nnz)}, err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat20",
                    choices=["rmat20", "stencil256", "uniform4096", "batched", "serve"])
    ap.add_argument("--rhs", type=int, default=0,
                    help="k > 0: time msrep_spmm with k right-hand sides (CSR) instead")
    ap.add_argument("--count", type=int, default=512, help="batched / serving pool size")
    ap.add_argument("--requests", type=int, default=2000, help="serving: requests per rate")
    ap.add_argument("--rates", default="0.1,0.5,0.9,1.2", help="serving: fractions of capacity")
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--vtype", default="f64", choices=["f64", "f32", "bf16"])
    ap.add_argument("--formats", default="csr,csc,coo")
    ap.add_argument("--nnz-per-wave", type=int, default=0, help="partition size (0: tuned)")
    ap.add_argument("--k", type=int, default=0)
    ap.add_argument("--wpb", type=int, default=0)
    ap.add_argument("--pipeline", type=int, default=0)
    ap.add_argument("--resident", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
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
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB copy (counter calibration)")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "KERNEL", "KEY"))
    ap.add_argument("--trace-summary", nargs=2, metavar=("TRACE_DIR", "OUT_NAME"))
    ap.add_argument("--command", default="", help="command line recorded in a summary")
    ap.add_argument("--bench-json", default=None, help="the traced run's output (trace summary)")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary, command=args.command)
        return 0
    if args.trace_summary:
        trace_summary(*args.trace_summary, command=args.command, bench_json=args.bench_json)
        return 0
    if args.gpus != 1:
        print("bench.py: one GPU only; --gpus %d is not supported (how the path would "
              "shard across GPUs is a design note, not code)" % args.gpus, file=sys.stderr)
        return 2

    import torch

    import paper_2209_07552_amd as pk
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    vt = {"f64": pk.F64, "f32": pk.F32, "bf16": pk.BF16}[args.vtype]
    if args.rhs > 0:
        return bench_spmm(args, vt)
    if args.workload == "batched":
        return bench_batched(args, vt)
    if args.workload == "serve":
        return bench_serve(args, vt)
    t0 = time.time()
    if args.workload == "rmat20":
        A, x64 = synth.rmat_csr(scale=20, edge_factor=16, seed=0)
        wl = {"workload": "rmat-scale20-ef16", "rows": A.m, "cols": A.n, "nnz": A.nnz,
              "abcd": [0.57, 0.19, 0.19, 0.05]}
    elif args.workload == "stencil256":
        A, x64 = synth.stencil7_csr(256, seed=0)
        wl = {"workload": "laplace3d-7pt-256^3", "rows": A.m, "cols": A.n, "nnz": A.nnz}
    else:
        A, x64 = synth.uniform_csr(4096, 4096, 16, seed=0)
        wl = {"workload": "uniform-4096-16perrow", "rows": A.m, "cols": A.n, "nnz": A.nnz}
    log("generated %s in %.1fs" % (wl["workload"], time.time() - t0))
    fmts = [f for f in args.formats.split(",") if f]
    H = host_formats(A, any_order="coo_any" in fmts)
    vbytes = pk._abi.VALUE_BYTES[vt]
    xbytes = 8 if vt == pk.F64 else 4

    def stored(v):
        if vt == pk.F64:
            return v
        v32 = np.asarray(v, np.float32)
        return v32 if vt == pk.F32 else synth.bf16_bits(v32)

    mats = {}
    for f in fmts:
        a, b, v = H[f]
        if f == "csr":
            mats[f] = pk.Mat(pk.CSR, vt, A.m, A.n, ptr=a, idx=b, val=stored(v))
        elif f == "csc":
            mats[f] = pk.Mat(pk.CSC, vt, A.m, A.n, ptr=a, idx=b, val=stored(v))
        else:
            kind = pk.COO_ANY if f == "coo_any" else pk.COO
            mats[f] = pk.Mat(kind, vt, A.m, A.n, idx=a, idx2=b, val=stored(v))
    if args.split != "rows":
        del H  # (the equal-rows baseline builds its partitions from it)
    xs = x64 if vt == pk.F64 else x64.astype(np.float32)
    x = torch.from_numpy(xs).to(dev)
    ydt = torch.float64 if vt == pk.F64 else torch.float32
    ys = {f: torch.zeros(A.m, dtype=ydt, device=dev) for f in fmts}
    # launch shape and partition size per format: explicit flags, else the
    # stored picks for this workload, else (or with --autotune) the tuner
    tunes, parts, part_ms = {}, {}, {}
    for f in fmts:
        stored_t = DEFAULT_TUNES.get(args.workload, {}).get(f)
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
            parts[f] = equal_rows_partition(mats[f], H, f, np_f, dev)
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

    def priced_of(kt):
        return {fk: v for fk, v in kt.items()
                if kernel_alg_bytes(fk[1], A.m, A.n, A.nnz, 1, vbytes, xbytes, fk[0]) is not None}

    def timed_steps(steps, only=None):
        """steps cold steps; each SpMV bracketed by events.  only=None: the
        library times every kernel; only=(fmt, kernel): just that kernel in
        that format's SpMV (one event pair, so the step is barely
        perturbed); only=False: no kernel timing."""
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
    # kernels whose algorithmic bytes are defined (the SpMV kernels proper)
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
    step_ms = sum(cold_ms.values())
    flops = 2.0 * A.nnz * len(fmts)
    per_fmt = {}
    for f in fmts:
        b = alg_bytes(f, A.m, A.n, A.nnz, vbytes, xbytes)
        each = sorted(a.elapsed_time(b) for a, b in ev[f])
        per_fmt[f] = {"ms_cold": round(cold_ms[f], 4),
                      "ms_cold_median": round(float(np.median(each)), 4),
                      "ms_cold_min": round(each[0], 4),
                      "gflops_cold": round(2.0 * A.nnz / cold_ms[f] / 1e6, 2),
                      "gbs_cold": round(b / cold_ms[f] / 1e6, 1),
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
    priced = priced_of(ktime)
    if not priced:  # no warmup: take the dominant kernel from the breakdown
        priced = priced_of(kt_all)
    (dom_f, kname), (kc, kt) = max(priced.items(), key=lambda kv: kv[1][1])
    k_ms = kt / kc
    k_bytes = kernel_alg_bytes(kname, A.m, A.n, A.nnz, parts[dom_f].np, vbytes, xbytes, dom_f)
    achieved = k_bytes / (k_ms * 1e-3) / 1e9
    traffic = load_traffic("%s/%s/%s" % (kname, wl["workload"], args.vtype))
    out = {
        "metric": "SpMV GFLOP/s (cold HBM; CSR+CSC+COO per step)",
        "value": round(flops / (step_ms * 1e-3) / 1e9, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(step_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.vtype, "data": "synthetic",
        "config": dict(wl, formats=fmts, value_type=args.vtype, split=args.split),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": kname, "format": dom_f,
                     "kernel_avg_us": round(k_ms * 1e3, 2), "alg_bytes_per_launch": int(k_bytes)},
        "per_format": per_fmt,
        "wall_s_timed_region": round(wall, 3),
    }
    if args.overheads:
        out["overheads"] = overheads(args, mats, part_ms, prep_ms, cold_ms, kt_all)
    if not args.no_cpu:
        f0 = "csr" if "csr" in fmts else fmts[0]
        yg = ys[f0].double().cpu().numpy()
        if vt == pk.F64:
            cb, err = cpu_baseline(A, x64, yg, args.cpu_budget)
            out["cpu_baseline"] = cb
            out["max_scaled_error_vs_oracle"] = err
        else:
            cb, err = cpu_baseline(A, x64, yg, args.cpu_budget)
            out["cpu_baseline"] = cb
            out["max_scaled_error_vs_fp64_oracle"] = err
    print(json.dumps(out), flush=True)
    return 0


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
    plain path (one msrep_spmv launch per matrix, same partitions)."""
    import torch

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
    tuned = {key: pk.msrep_autotune(Ms[k], xs[k]) for key, k in classes.items()}
    tunes = [pk.Tune(k_per_lane=4, waves_per_wg=4,
                     nnz_per_wave=tuned[(k % 2, int(np.log10(max(A.m, 10))))].nnz_per_wave)
             for k, (A, _) in enumerate(mats)]
    log("autotuned %d classes in %.1fs" % (len(classes), time.time() - t0))
    plan = pk.msrep_plan_create(Ms, tunes)
    for _ in range(args.warmup):
        pk.msrep_spmv_batched(plan, xs, ys)
    ms_b = _timed(lambda: pk.msrep_spmv_batched(plan, xs, ys), args.steps)
    # plain path: one launch (plus merge) per matrix
    parts = [pk.msrep_build_partition(M, max(1, -(-M.nnz // t.nnz_per_wave))) for M, t in zip(Ms, tunes)]
    ws = torch.zeros(1 << 26, dtype=torch.uint8, device=dev)

    def plain():
        for M, P, x, y, t in zip(Ms, parts, xs, ys, tunes):
            pk.msrep_spmv(M, P, x, y, 1.0, 0.0, t, ws=ws)
    for _ in range(args.warmup):
        plain()
    ms_p = _timed(plain, max(1, args.steps // 4))
    out = {"metric": "batched SpMV/s (%d uneven matrices, one persistent hipGraph launch)" % args.count,
           "value": round(args.count / (ms_b * 1e-3), 1), "unit": "SpMV/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_b, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.vtype,
           "data": "synthetic",
           "config": {"workload": "batched-%d" % args.count, "total_nnz": nnz, "items": plan.items()},
           "gflops": round(2.0 * nnz / (ms_b * 1e-3) / 1e9, 2),
           "alg_gbs": round(byts / (ms_b * 1e-3) / 1e9, 1),
           "plain_path": {"ms_per_batch": round(ms_p, 4),
                          "spmv_per_s": round(args.count / (ms_p * 1e-3), 1)},
           "speedup_vs_plain": round(ms_p / ms_b, 3)}
    print(json.dumps(out), flush=True)
    return 0


def bench_serve(args, vt):
    """Poisson request stream over a pool of batched-style matrices; each
    request = one matrix + 10..100 SpMVs with fresh x; arena budget as given.
    Rates are fractions of the measured batched capacity.  Beside it, the
    plain FP64 path: one request at a time, one msrep_spmv launch per SpMV."""
    import torch

    import paper_2209_07552_amd as pk
    from paper_2209_07552_amd import serving
    import synth
    dev = torch.device("cuda:0")
    t0 = time.time()
    pool = [A for A, _ in synth.batched_set(args.count, seed=0)]
    log("generated pool of %d in %.1fs" % (len(pool), time.time() - t0))
    mean_steps = 55.0
    # capacity estimate from a saturated run: SpMVs per second of the mix
    probe = synth.serving_trace(max(64, args.count // 4), rate=1e9, pool=len(pool), seed=99)
    _, st = serving.serve(pool, probe, budget_bytes=int(args.budget_gb * (1 << 30)), vtype=vt,
                          max_slots=256)
    cap_req = st["spmv_per_s"] / mean_steps
    log("saturated mix: %.0f SpMV/s -> capacity ~%.1f req/s" % (st["spmv_per_s"], cap_req))
    points = []
    for f in [float(v) for v in args.rates.split(",")]:
        trace = synth.serving_trace(args.requests, rate=max(f * cap_req, 1e-3), pool=len(pool), seed=1)
        _, st = serving.serve(pool, trace, budget_bytes=int(args.budget_gb * (1 << 30)), vtype=vt,
                              max_slots=256)
        points.append({"load": f, "rate_req_s": round(f * cap_req, 2),
                       "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
                       "req_per_s": round(st["req_per_s"], 2),
                       "spmv_per_s": round(st["spmv_per_s"], 1), "gflops": round(st["gflops"], 2),
                       "peak_active": st["peak_active"], "ticks": st["ticks"]})
        log(json.dumps(points[-1]))
    # plain FP64 path: requests one after another, one launch per SpMV
    sample = synth.serving_trace(64, rate=1.0, pool=len(pool), seed=1)
    ws = torch.zeros(1 << 26, dtype=torch.uint8, device=dev)
    lat = []
    for q in sample:
        A = pool[q.matrix]
        M = pk.Mat(pk.CSR, pk.F64, A.m, A.n, ptr=A.ptr, idx=A.col, val=A.val)
        P = pk.msrep_build_partition(M, max(1, -(-A.nnz // 1024)))
        x = torch.empty(A.n, dtype=torch.float64, device=dev)
        y = torch.empty(A.m, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for j in range(q.steps):
            x.copy_(torch.from_numpy(synth.serving_x(A.n, 0, q.rid, j)), non_blocking=False)
            pk.msrep_spmv(M, P, x, y, ws=ws)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
    best = max(points, key=lambda p: p["req_per_s"])
    out = {"metric": "served p50/p99 latency and req/s (Poisson, continuous batching)",
           "value": best["req_per_s"], "unit": "req/s", "n_gpus": 1, "steps": args.requests,
           "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": args.vtype, "data": "synthetic",
           "config": {"workload": "serve-pool%d" % len(pool), "budget_gb": args.budget_gb,
                      "steps_per_request": "U{10..100}"},
           "points": points,
           "plain_fp64_one_request_at_a_time": {
               "p50_ms": round(float(np.percentile(lat, 50)), 3),
               "p99_ms": round(float(np.percentile(lat, 99)), 3),
               "req_per_s": round(1e3 / float(np.mean(lat)), 2),
               "note": "service time only (no queueing); x generated on the host per step"}}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
