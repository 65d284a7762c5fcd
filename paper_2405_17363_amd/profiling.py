"""Summaries of rocprofv3 output for the solve kernels.

    python -m paper_2405_17363_amd.profiling stats  --trace DIR [--kernel NAME] [--last N]
    python -m paper_2405_17363_amd.profiling traffic --fetch DIR --write DIR --ncells C --lanes L --out FILE
    python -m paper_2405_17363_amd.profiling counters --pmc DIR [--pmc DIR ...] --kernel NAME [--last N]

The traffic summary is a text file: '#' lines describe how it was made, the
rest is one JSON object (read back with ``load_traffic``).

``traffic`` reads two ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs (CSV
output) of ``bench.py --copy-calibration``.  That run first copies a 1 GiB
device buffer; the counters' readings for that copy (2^30 bytes read and
2^30 bytes written) give the factor that turns counter units into bytes, and
the same factors scale the solve kernel's readings.  The result records a
hash of the kernel sources, so that a later benchmark can tell whether the
kernel has changed since the counters were taken.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 1 << 30


def source_hash() -> str:
    """Hash of the kernel and host sources of the library."""
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))):
        with open(path, "rb") as f:
            h.update(os.path.basename(path).encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def _csv(dirname: str, suffix: str):
    paths = glob.glob(os.path.join(dirname, "**", "*" + suffix), recursive=True)
    if not paths:
        raise FileNotFoundError(f"no *{suffix} under {dirname}")
    with open(paths[0]) as f:
        return list(csv.DictReader(f))


def _is(name: str, kernel: str) -> bool:
    """`name` (as rocprofv3 prints it) is `kernel`: the same name, or a
    demangled C++ name whose function is `kernel`."""
    return name == kernel or ("::" + kernel + "(") in name or name.startswith(kernel + "(")


def kernel_stats(trace_dir: str, kernel: str = "bcs_solve_fp64", last: int = 0, drop_last: int = 0) -> dict:
    """rocprofv3's statistics for `kernel`; with last > 0 also the mean
    duration of its last `last` dispatches (the timed ones after a warm-up),
    leaving out the final `drop_last` dispatches (launches made after the
    timed ones, such as the cache-flushed calls of bench.py)."""
    for r in _csv(trace_dir, "kernel_stats.csv"):
        if _is(r["Name"], kernel):
            out = {"kernel": kernel, "calls": int(r["Calls"]), "avg_ns": float(r["AverageNs"]),
                   "min_ns": float(r["MinNs"]), "max_ns": float(r["MaxNs"])}
            if last > 0:
                d = [(int(t["Start_Timestamp"]), int(t["End_Timestamp"]) - int(t["Start_Timestamp"]))
                     for t in _csv(trace_dir, "kernel_trace.csv") if _is(t["Kernel_Name"], kernel)]
                d = [ns for _, ns in sorted(d)]
                d = d[:len(d) - drop_last][-last:]
                out["last"] = len(d)
                out["last_avg_ns"] = sum(d) / len(d)
            return out
    raise KeyError(kernel)


def per_dispatch(pmc_dir: str, counter: str) -> list:
    """[(kernel name, grid size, summed counter value)] in dispatch order."""
    acc = collections.OrderedDict()
    for r in _csv(pmc_dir, "counter_collection.csv"):
        if r["Counter_Name"] != counter:
            continue
        key = (int(r["Dispatch_Id"]), r["Kernel_Name"], int(r["Grid_Size"]))
        acc[key] = acc.get(key, 0.0) + float(r["Counter_Value"])
    return [(k[1], k[2], v) for k, v in sorted(acc.items())]


def counters(pmc_dirs, kernel: str, last: int = 0, drop_last: int = 0) -> dict:
    """Mean per dispatch of every counter in the `--pmc` runs `pmc_dirs` for
    `kernel` (each dispatch's value summed over instances), over its last
    `last` dispatches (all if 0) once the final `drop_last` are left out."""
    out = {}
    for d in pmc_dirs:
        names = sorted({r["Counter_Name"] for r in _csv(d, "counter_collection.csv")})
        for c in names:
            v = [val for name, g, val in per_dispatch(d, c) if _is(name, kernel)]
            v = v[:len(v) - drop_last]
            if last > 0:
                v = v[-last:]
            if v:
                out[c] = sum(v) / len(v)
                out.setdefault("_dispatches", len(v))
    return out


def traffic(fetch_dir: str, write_dir: str, kernel: str = "bcs_solve_fp64", last: int = 0,
            drop_last: int = 0) -> dict:
    """HBM bytes per launch of `kernel` (mean over its last `last` dispatches,
    all if 0, once the final `drop_last` are left out) from a FETCH_SIZE and
    a WRITE_SIZE run of `bench.py --copy-calibration`."""
    f = per_dispatch(fetch_dir, "FETCH_SIZE")
    w = per_dispatch(write_dir, "WRITE_SIZE")
    # the calibration copy is the copy kernel with the largest write
    copy_w = max((v for name, g, v in w if "copyBuffer" in name), default=0.0)
    copy_f = max((v for name, g, v in f if "copyBuffer" in name), default=0.0)
    if copy_w <= 0 or copy_f <= 0:
        raise RuntimeError("calibration copy not found in the counter runs")
    kf = COPY_BYTES / copy_f
    kw = COPY_BYTES / copy_w
    fk = [v for name, g, v in f if _is(name, kernel)]
    wk = [v for name, g, v in w if _is(name, kernel)]
    fk, wk = fk[:len(fk) - drop_last], wk[:len(wk) - drop_last]
    if last > 0:
        fk, wk = fk[-last:], wk[-last:]
    if not fk or not wk:
        raise RuntimeError(f"{kernel} not found in the counter runs")
    fetch = kf * sum(fk) / len(fk)
    write = kw * sum(wk) / len(wk)
    return {"kernel": kernel, "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
            "hbm_bytes_per_launch": fetch + write, "fetch_factor": kf, "write_factor": kw,
            "launches": len(fk), "source_hash": source_hash()}


def measure_peaks(reps: int = 5) -> dict:
    """Attained ceilings on the current device (include/bcs_probe.h): HBM
    stream (a 1 GiB copy), LDS gathers of FP64 words (conflict-free and
    pseudo-random), FP64 and FP32 vector FMAs.  Each probe is launched once
    untimed, then `reps` times, each timed with HIP events on the current
    stream; the best rate is kept."""
    import ctypes

    import torch

    from ._binding import lib

    L = lib()
    dev = torch.cuda.current_device()
    cu = torch.cuda.get_device_properties(dev).multi_processor_count
    stream = torch.cuda.current_stream()
    sh = ctypes.c_void_p(stream.cuda_stream)
    threads = L.bcs_probe_threads_per_block()

    def best(launch):
        if launch() < 0:
            raise RuntimeError("probe launch failed")
        out = 0.0
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            amount = launch()
            e1.record(stream)
            e1.synchronize()
            out = max(out, amount / (e0.elapsed_time(e1) * 1e-3))
        return out

    n = 1 << 27  # 1 GiB of FP64 each way
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    blocks = cu * 16
    hbm = best(lambda: L.bcs_probe_copy(a.data_ptr(), b.data_ptr(), n, blocks, sh))
    del a, b
    blocks = cu * 8
    sink = torch.empty(blocks * threads, dtype=torch.float64, device=dev)
    lds0 = best(lambda: L.bcs_probe_lds(sink.data_ptr(), 2000, 0, blocks, sh))
    lds1 = best(lambda: L.bcs_probe_lds(sink.data_ptr(), 2000, 1, blocks, sh))
    f64 = best(lambda: L.bcs_probe_fma(sink.data_ptr(), 5000, 1, blocks, sh))
    sink32 = torch.empty(blocks * threads, dtype=torch.float32, device=dev)
    f32 = best(lambda: L.bcs_probe_fma(sink32.data_ptr(), 5000, 0, blocks, sh))
    torch.cuda.synchronize()
    return {"hbm_copy_gbs": round(hbm / 1e9, 1), "lds_gather_tbs": round(lds0 / 1e12, 2),
            "lds_random_gather_tbs": round(lds1 / 1e12, 2), "fp64_fma_tflops": round(f64 / 1e12, 2),
            "fp32_fma_tflops": round(f32 / 1e12, 2), "compute_units": cu,
            "how": "include/bcs_probe.h kernels, best of %d event-timed launches each" % reps}


def load_traffic(path: str) -> dict:
    with open(path) as f:
        return json.loads("".join(line for line in f if not line.lstrip().startswith("#")))


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--trace", required=True)
    s.add_argument("--kernel", default="bcs_solve_fp64")
    s.add_argument("--last", type=int, default=0, help="also average the last N dispatches")
    s.add_argument("--drop-last", type=int, default=0, help="leave out the final N dispatches")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", default="bcs_solve_fp64")
    t.add_argument("--ncells", type=int, required=True)
    t.add_argument("--lanes", type=int, required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--last", type=int, default=0, help="average the last N dispatches only")
    t.add_argument("--drop-last", type=int, default=0, help="leave out the final N dispatches")
    t.add_argument("--note", action="append", default=[], help="header line for the summary (repeatable)")
    c = sub.add_parser("counters")
    c.add_argument("--pmc", action="append", required=True, help="a --pmc run's output directory (repeatable)")
    c.add_argument("--kernel", default="bcs_solve_fp64")
    c.add_argument("--last", type=int, default=0)
    c.add_argument("--drop-last", type=int, default=0, help="leave out the final N dispatches")
    a = ap.parse_args(argv)
    if a.cmd == "counters":
        print(json.dumps(counters(a.pmc, a.kernel, a.last, a.drop_last)))
        return 0
    if a.cmd == "stats":
        print(json.dumps(kernel_stats(a.trace, a.kernel, a.last, a.drop_last)))
        return 0
    res = traffic(a.fetch, a.write, a.kernel, a.last, a.drop_last)
    res.update({"ncells": a.ncells, "lanes_per_cell": a.lanes})
    with open(a.out, "w") as f:
        for line in a.note:
            f.write("# " + line + "\n")
        json.dump(res, f, indent=1)
        f.write("\n")
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
