"""Benchmark: cell-systems solved per second at relative residual 1e-10.

Workload: 100,000 cells of the synthetic n = 80 mass-action mechanism (150
reactions), h log-uniform in [1e-3, 100] s (gamma = h/2), b ~ N(0, 1), Jacobi
right preconditioning, rtol 1e-10, maxit 200.  A step is one batched FP64
Block-cells BiCGStab solve of all cells (stage A = I - gamma J, iterate,
confirm the true residual, write x / iterations / residuals / statuses), with
every input already resident in device memory.  The FP32-inner /
FP64-refinement form is timed on the same inputs and reported beside it.

Prints ONE JSON line.  Only one GPU is used: --gpus above 1 exits.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "cell-systems solved/s at rel. residual 1e-10, 100k cells (FP64 vs FP32+refine)"
HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, GB/s
FP64_VALU_PEAK = 78.6     # MI355X FP64 vector, TFLOP/s
LDS_PEAK_TBS = 128 * 256 * 2.4e9 / 1e12  # 128 B per clock per CU, 256 CUs, 2.4 GHz: 78.6 TB/s
FP32_VALU_PEAK = 157.3    # MI355X FP32 vector (packed FMA), TFLOP/s
FP32_UNPACKED_PEAK = 78.6  # FP32 vector without packed instructions (what the kernels issue), TFLOP/s
RTOL = 1e-10
MAXIT = 200
FORMS = ("mixed", "mixed_cell", "adjoint", "multi", "block", "ilu0", "assemble", "mech", "small", "peaks")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # about 20 ms of untimed work: the GPU's clocks ramp up over the first
    # launches, and shorter warm-ups time the ramp
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--ncells", type=int, default=100_000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--forms", default="all",
                    help="comma list of the forms timed beside the headline solve: " + ",".join(FORMS) +
                         ", or 'all' / 'none'")
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--cell-order", type=int, default=1, choices=(0, 1),
                    help="1: cells handed out in the cost order (sorted by gamma on the device each step)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy a 1 GiB device buffer (reference for HBM byte counters)")
    a = ap.parse_args()
    a.forms = set(FORMS) if a.forms == "all" else set() if a.forms == "none" else set(a.forms.split(","))
    unknown = a.forms - set(FORMS)
    if unknown:
        ap.error("unknown forms: " + ",".join(sorted(unknown)))
    return a


def algorithmic_bytes_per_cell(n: int, nnz: int) -> int:
    # read J values, b, gamma; write x, resid, iters, status (A stays on chip)
    return 8 * nnz + 8 * n + 8 + 8 * n + 8 + 4 + 4


def flops_per_cell(n: int, nnz: int, iters: np.ndarray, status: np.ndarray) -> float:
    # per full iteration: 2 SpMV (2*nnz FMA each) + 6 dots/norms + 4 vector
    # updates = 4 nnz + 24 n; staging (form A, column scaling, ||b||) and the
    # true-residual check = about 3 nnz + 7 n + (2 nnz + 3 n) per confirmation
    it = iters.astype(np.float64)
    return float(np.sum(it * (4 * nnz + 24 * n) + (5 * nnz + 10 * n)))


def roofline(kernel: str, seconds: float, hbm_bytes: float, flops: float, lds_bytes: float,
             valu_peak: float = FP64_VALU_PEAK, traffic=None, **extra) -> dict:
    """Fractions of the three ceilings the solve can exhaust (HBM bytes,
    vector FLOPs, LDS operand gathers) for one launch's algorithmic work over
    its measured duration; `bound` is the binding one, the largest fraction."""
    ach = {"hbm": hbm_bytes / seconds / 1e9, "alu": flops / seconds / 1e12, "lds": lds_bytes / seconds / 1e12}
    peak = {"hbm": HBM_PEAK_GBS, "alu": valu_peak, "lds": LDS_PEAK_TBS}
    unit = {"hbm": "GB/s", "alu": "TFLOP/s", "lds": "TB/s"}
    frac = {k: ach[k] / peak[k] for k in ach}
    bound = max(frac, key=frac.get)
    out = {"bound": bound, "achieved": round(ach[bound], 3), "peak": peak[bound], "unit": unit[bound],
           "frac": round(frac[bound], 4), "traffic": traffic, "kernel": kernel,
           "avg_launch_ms": round(seconds * 1e3, 4),
           "hbm_gbs": round(ach["hbm"], 2), "hbm_frac": round(frac["hbm"], 4),
           "valu_tflops": round(ach["alu"], 3), "valu_peak": valu_peak, "valu_frac": round(frac["alu"], 4),
           "lds_gather_tbs": round(ach["lds"], 2), "lds_gather_frac": round(frac["lds"], 4),
           "algorithmic_bytes_per_launch": hbm_bytes, "algorithmic_flops_per_launch": flops,
           "lds_gather_bytes_per_launch": lds_bytes}
    out.update(extra)
    return out


def ilu_counts(row_ptr, col_idx):
    """Entries of the strict lower and upper triangles of the pattern, and the
    flops of one ILU(0) factorisation on it (IKJ: a division per lower entry,
    an FMA per update a_ij -= l_ik u_kj with (i, j) in the pattern)."""
    n = len(row_ptr) - 1
    rows = [set(col_idx[row_ptr[i]:row_ptr[i + 1]].tolist()) for i in range(n)]
    zl = sum(1 for i in range(n) for j in rows[i] if j < i)
    zu = sum(1 for i in range(n) for j in rows[i] if j > i)
    fl = 0
    for i in range(n):
        for k in sorted(j for j in rows[i] if j < i):
            fl += 1 + 2 * sum(1 for j in rows[k] if j > k and j in rows[i])
    return zl, zu, fl


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import paper_2405_17363_amd as bcs
    from workload import config_inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    t0 = time.time()
    mech, cells = config_inputs(3, ncells=None if args.ncells == 100_000 else args.ncells)[0]
    C, n, nnz = cells["b"].shape[0], mech.n, mech.nnz
    print(f"# generated {C} cells n={n} nnz={nnz} in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    if args.copy_calibration:
        # a plain device-to-device copy of known size: 2^30 bytes read, 2^30 written
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    values = torch.as_tensor(cells["values"], device=dev)
    gamma = torch.as_tensor(cells["gamma"], device=dev)
    b = torch.as_tensor(cells["b"], device=dev)
    plan = bcs.Plan(mech.row_ptr, mech.col_idx, precond="jacobi", lanes_per_cell=args.lanes,
                    cell_order=bool(args.cell_order))
    if args.lanes == 0:
        # the library's autotuner on this batch (outside the timed region)
        plan.autotune(values, gamma, b, RTOL, MAXIT)
    out = [torch.empty((C, n), dtype=torch.float64, device=dev), torch.empty(C, dtype=torch.int32, device=dev),
           torch.empty(C, dtype=torch.float64, device=dev), torch.empty(C, dtype=torch.int32, device=dev),
           torch.empty(C, dtype=torch.int32, device=dev)]
    stream = torch.cuda.current_stream()
    ws = plan.workspace(C, dev)

    def step():
        bcs.solve_batch(plan, values, gamma, b, RTOL, MAXIT, out=out, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # per-launch durations with events on the launch stream
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        step()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    kern_ms = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
    ms_per_step = 1e3 * wall / args.steps
    x, iters, resid, status, _ = [t.cpu().numpy() for t in out]
    solved = int(np.sum((status == 0) & (resid <= RTOL)))
    value = solved / (ms_per_step * 1e-3)
    avg_launch_s = float(np.mean(kern_ms)) * 1e-3
    bytes_launch = algorithmic_bytes_per_cell(n, nnz) * C
    flops_launch = flops_per_cell(n, nnz, iters, status)
    info = plan.info()

    # HBM bytes per launch from the committed counter summary, used only while
    # the kernel sources and the layout are those the counters were taken with
    traffic = None
    tr_path = os.path.join(HERE, "profiles", "traffic_fp64_solve_100k_n80.txt")
    if os.path.exists(tr_path):
        from paper_2405_17363_amd.profiling import load_traffic, source_hash

        tr = load_traffic(tr_path)
        if (tr.get("source_hash") == source_hash() and tr.get("ncells") == C
                and tr.get("lanes_per_cell") == info["lanes_per_cell"]):
            traffic = round(tr["hbm_bytes_per_launch"])

    # on-chip operand gathers: every stored entry gathers one FP64 operand per
    # SpMV (two per iteration, one for staging's column scaling, one for the
    # true residual)
    lds_bytes = float(np.sum(iters.astype(np.float64) * 16 * nnz + 16 * nnz))
    roofline_obj = roofline(
        "bcs_solve_fp64 (%d lanes/cell, %d rows/lane, %d steps/lane)" % (
            info["lanes_per_cell"], info["rows_per_lane"], info["steps_per_lane"]),
        avg_launch_s, bytes_launch, flops_launch, lds_bytes, traffic=traffic)

    # the same launch after a 1 GiB scratch write (no input left in the L2 or
    # the Infinity Cache): per-call event times only, not the headline
    scratch = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    flushed = []
    for _ in range(min(args.steps, 10)):
        scratch.fill_(1.0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        step()
        e1.record(stream)
        torch.cuda.synchronize()
        flushed.append(e0.elapsed_time(e1))
    del scratch
    roofline_obj["avg_launch_ms_after_cache_flush"] = round(float(np.mean(flushed)), 4)

    # Unsolved cells whose FP64 evaluation floor is above rtol: the relative
    # residual of their dense-LU solution (numpy, FP64) exceeds rtol / 2, so
    # no FP64 method can report them within rtol ("floor-limited"; they are
    # never counted as solved).
    lu_rows = np.repeat(np.arange(n), np.diff(mech.row_ptr))

    def floor_limited_count(unsolved_cells, rhs, transpose=False):
        count = 0
        for c in unsolved_cells:
            A = np.zeros((n, n))
            A[lu_rows, mech.col_idx] = -cells["gamma"][c] * cells["values"][c]
            A[np.arange(n), np.arange(n)] += 1.0
            if transpose:
                A = A.T.copy()
            xl = np.linalg.solve(A, rhs[c])
            rho = np.linalg.norm(rhs[c] - A @ xl) / np.linalg.norm(rhs[c])
            count += int(rho > RTOL / 2)
        return count

    floor_limited = floor_limited_count(np.nonzero(~((status == 0) & (resid <= RTOL)))[0], cells["b"])

    def mixed_form(budget):
        try:
            mplan = bcs.Plan(mech.row_ptr, mech.col_idx, precond="jacobi", precision="fp32_refine",
                             lanes_per_cell=args.lanes, cell_order=bool(args.cell_order), refine_budget=budget)
            if args.lanes == 0:
                mplan.autotune(values, gamma, b, RTOL, MAXIT)
            mout = [torch.empty_like(o) for o in out]

            def mstep():
                bcs.solve_batch(mplan, values, gamma, b, RTOL, MAXIT, out=mout, workspace=ws)

            for _ in range(args.warmup):
                mstep()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                mstep()
            torch.cuda.synchronize()
            mms = 1e3 * (time.perf_counter() - t1) / args.steps
            mx, mit, mres, mst, mref = [t.cpu().numpy() for t in mout]
            msolved = int(np.sum((mst == 0) & (mres <= RTOL)))
            both = (mst == 0) & (status == 0)
            err = np.linalg.norm(mx[both] - x[both], axis=1) / np.linalg.norm(x[both], axis=1)
            # FP32 inner iterations (two SpMVs, six reductions, four updates) plus
            # FP64 work: staging (form A, scale, cast) and per refinement the
            # residual b - A x, its norm and the update x += ||r|| D^-1 d
            mi = mit.astype(np.float64)
            mr = mref.astype(np.float64)
            f32 = float(np.sum(mi * (4 * nnz + 24 * n)))
            f64 = float(np.sum(mr * (2 * nnz + 8 * n) + (4 * nnz + 6 * n)))
            # gathers: 4-byte FP32 operands in the inner solve, 8-byte FP64 in
            # the residual of every refinement and in staging's scaling
            mlds = float(np.sum(mi * 8 * nnz + mr * 8 * nnz + 8 * nnz))
            mroof = roofline("bcs_solve_mixed (%d lanes/cell)" % mplan.info()["lanes_per_cell"], mms * 1e-3,
                             algorithmic_bytes_per_cell(n, nnz) * C, f32 + f64, mlds, valu_peak=FP32_VALU_PEAK,
                             fp32_flops_per_launch=f32, fp64_flops_per_launch=f64,
                             valu_frac_unpacked=round((f32 + f64) / (mms * 1e-3) / 1e12 / FP32_UNPACKED_PEAK, 4))
            return {"value": round(msolved / (mms * 1e-3), 1), "ms_per_step": round(mms, 4), "roofline": mroof,
                    "refine_budget": budget, "lanes_per_cell": mplan.info()["lanes_per_cell"],
                    "solved_fraction": round(msolved / C, 5), "iters_mean": round(float(mit.mean()), 2),
                    "refinements_mean": round(float(mref.mean()), 3),
                    "unsolved_floor_limited": floor_limited_count(
                        np.nonzero(~((mst == 0) & (mres <= RTOL)))[0], cells["b"]),
                    "rel_diff_vs_fp64_max": float(err.max()) if err.size else None,
                    "rel_diff_vs_fp64_p99": float(np.percentile(err, 99)) if err.size else None}
        except bcs.BcsError as e:
            return {"error": str(e)}

    mixed = mixed_cell = None
    if "mixed" in args.forms:
        mixed = mixed_form("inner")
    if "mixed_cell" in args.forms:
        mixed_cell = mixed_form("cell")

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    adjoint = multi = block_cells = None
    if "adjoint" in args.forms:
        # adjoint of the same batch: lambda = A^-T g (g ~ N(0,1)), dL/dA on the pattern
        g_host = np.random.default_rng(7).standard_normal((C, n))
        g = torch.as_tensor(g_host, device=dev)
        xf = out[0].clone()
        res_adj = {}

        def astep():
            res_adj["r"] = bcs.solve_batch_adjoint(plan, values, gamma, xf, g, RTOL, MAXIT, workspace=ws)

        ams = timed(astep, args.steps)
        ast = res_adj["r"][5].cpu().numpy()
        ares = res_adj["r"][4].cpu().numpy()
        asolved = int(np.sum((ast == 0) & (ares <= RTOL)))
        adjoint = {"value": round(asolved / (ams * 1e-3), 1), "unit": "cells/s", "ms_per_step": round(ams, 4),
                   "solved_fraction": round(asolved / C, 5),
                   "iters_mean": round(float(res_adj["r"][3].float().mean().item()), 2),
                   "unsolved_floor_limited": floor_limited_count(np.nonzero(~((ast == 0) & (ares <= RTOL)))[0],
                                                                 g_host, transpose=True),
                   "algorithmic_bytes_per_cell": 16 * nnz + 24 * n + 32}
        ait = res_adj["r"][3].cpu().numpy().astype(np.float64)
        adjoint["roofline"] = roofline(
            "bcs_solve_adjoint (%d lanes/cell)" % info["lanes_per_cell"], ams * 1e-3,
            (16 * nnz + 24 * n + 32) * C,
            # the transposed solve's iterations and staging, then dL/dA = -lambda_i x_j
            float(np.sum(ait * (4 * nnz + 24 * n) + (5 * nnz + 10 * n) + nnz)),
            float(np.sum(ait * 16 * nnz + 16 * nnz)))
        del g, xf, res_adj
    if "multi" in args.forms:
        # three mechanisms (n = 30 / 80 / 200, 12.5k / 25k / 12.5k cells) in one persistent launch,
        # against the same cells solved by one launch per mechanism
        mechs = config_inputs(4)
        MV = [torch.as_tensor(c["values"], device=dev) for _, c in mechs]
        MG = [torch.as_tensor(c["gamma"], device=dev) for _, c in mechs]
        MB = [torch.as_tensor(c["b"], device=dev) for _, c in mechs]
        # the combined launch runs at the occupancy of its heaviest mechanism, so its lane
        # counts are tuned on the combined launch; the separate launches each tune alone
        mplans = [bcs.Plan(m.row_ptr, m.col_idx, precond="jacobi") for m, _ in mechs]
        eplans = [bcs.Plan(m.row_ptr, m.col_idx, precond="jacobi") for m, _ in mechs]
        bcs.multi_autotune(mplans, MV, MG, MB, RTOL, MAXIT)
        for pl, v, gg, bb in zip(eplans, MV, MG, MB):
            pl.autotune(v, gg, bb, RTOL, MAXIT)
        res_m = {}

        def mstep_multi():
            res_m["r"] = bcs.solve_multi(mplans, MV, MG, MB, RTOL, MAXIT)

        def mstep_each():
            for pl, v, gg, bb in zip(eplans, MV, MG, MB):
                bcs.solve_batch(pl, v, gg, bb, RTOL, MAXIT)

        mms = timed(mstep_multi, args.steps)
        ems = timed(mstep_each, args.steps)
        mc = sum(int(v.shape[0]) for v in MV)
        msolved = sum(int(np.sum((r[3].cpu().numpy() == 0) & (r[2].cpu().numpy() <= RTOL))) for r in res_m["r"])
        mbytes = sum(algorithmic_bytes_per_cell(m.n, m.nnz) * int(v.shape[0]) for (m, _), v in zip(mechs, MV))
        mflops = sum(flops_per_cell(m.n, m.nnz, r[1].cpu().numpy(), r[3].cpu().numpy())
                     for (m, _), r in zip(mechs, res_m["r"]))
        mlds = sum(float(np.sum(r[1].cpu().numpy().astype(np.float64) * 16 * m.nnz + 16 * m.nnz))
                   for (m, _), r in zip(mechs, res_m["r"]))
        multi = {"value": round(msolved / (mms * 1e-3), 1), "unit": "cells/s", "ms_per_step": round(mms, 4),
                 "roofline": roofline("bcs_solve_multi (%s lanes/cell)" % "/".join(
                     str(pl.info()["lanes_per_cell"]) for pl in mplans), mms * 1e-3, mbytes, mflops, mlds),
                 "ncells": mc, "solved_fraction": round(msolved / mc, 5),
                 "ms_one_launch_per_mechanism": round(ems, 4),
                 "lanes_per_cell": [pl.info()["lanes_per_cell"] for pl in mplans],
                 "lanes_per_cell_one_launch_per_mechanism": [pl.info()["lanes_per_cell"] for pl in eplans]}
        del MV, MG, MB, res_m
    if "block" in args.forms:
        # Block-cells (N) of Section 3 against Block-cells (1) on the same batch: the cells of a wave
        # (64 / lanes consecutive cells) solved as one block-diagonal system with shared scalars
        block_cells = []
        for L in (32, 16):
            row = {"lanes_per_cell": L, "cells_per_run": 64 // L}
            for key, shared in (("bc1", False), ("bcN", True)):
                bplan = bcs.Plan(mech.row_ptr, mech.col_idx, precond="jacobi", lanes_per_cell=L,
                                 shared_scalars=shared, cell_order=not shared)
                bout = [torch.empty_like(o) for o in out]

                def bstep(bplan=bplan, bout=bout):
                    bcs.solve_batch(bplan, values, gamma, b, RTOL, MAXIT, out=bout)

                bms = timed(bstep, args.steps)
                bit, bres, bst = bout[1].cpu().numpy(), bout[2].cpu().numpy(), bout[3].cpu().numpy()
                bsolved = int(np.sum((bst == 0) & (bres <= RTOL)))
                G = 64 // L if shared else 1
                runs = bit[: (C // G) * G].reshape(-1, G)
                row[key] = {"value": round(bsolved / (bms * 1e-3), 1), "ms_per_step": round(bms, 4),
                            "solved_fraction": round(bsolved / C, 5),
                            "iters_mean_per_run": round(float(runs[:, 0].mean()), 2),
                            "iters_max": int(bit.max()),
                            "run_iters_over_slowest_cell": None}
                if shared:
                    one = row["bc1"]["_iters"][: (C // G) * G].reshape(-1, G).max(axis=1)
                    row[key]["run_iters_over_slowest_cell"] = round(float(np.mean(runs[:, 0] / one)), 3)
                else:
                    row[key]["_iters"] = bit
                del bplan, bout
            row["bc1"].pop("_iters")
            block_cells.append(row)

    # ILU(0) right preconditioning (the stronger preconditioner the paper
    # names as its next optimisation) on the same 100k cells
    ilu = None
    if "ilu0" in args.forms:
        try:
            iplan = bcs.Plan(mech.row_ptr, mech.col_idx, precond="ilu0", cell_order=bool(args.cell_order))
            iplan.autotune(values, gamma, b, RTOL, MAXIT)
            iout = [torch.empty_like(o) for o in out]

            def istep():
                bcs.solve_batch(iplan, values, gamma, b, RTOL, MAXIT, out=iout, workspace=ws)

            ims = timed(istep, args.steps)
            ix, iit, ires, ist, _ = [t.cpu().numpy() for t in iout]
            isolved = int(np.sum((ist == 0) & (ires <= RTOL)))
            zl, zu, ffl = ilu_counts(mech.row_ptr, mech.col_idx)
            sw = iplan.options.ilu_sweeps or 3  # 0 = the library default, 3 sweeps
            ii = iit.astype(np.float64)
            # per iteration: two SpMVs with A, two applications of (LU)^-1 by
            # `sw` sweeps per triangle, six reductions and four updates; per
            # cell: forming A, the factorisation and the true residual
            per_it = 4 * nnz + 24 * n + 2 * (sw * (2 * zl + n) + n + sw * (2 * zu + n))
            iflops = float(np.sum(ii * per_it + ffl + 5 * nnz + 10 * n))
            ilds = float(np.sum(ii * 8 * (2 * nnz + 2 * sw * (zl + zu)) + 8 * (zl + zu + nnz)))
            both = (ist == 0) & (status == 0)
            err = np.linalg.norm(ix[both] - x[both], axis=1) / np.linalg.norm(x[both], axis=1)
            ilu = {"value": round(isolved / (ims * 1e-3), 1), "unit": "cells/s", "ms_per_step": round(ims, 4),
                   "solved_fraction": round(isolved / C, 5), "iters_mean": round(float(iit.mean()), 2),
                   "iters_p99": float(np.percentile(iit, 99)), "iters_max": int(iit.max()), "sweeps": sw,
                   "lanes_per_cell": iplan.info()["lanes_per_cell"],
                   "unsolved_floor_limited": floor_limited_count(np.nonzero(~((ist == 0) & (ires <= RTOL)))[0],
                                                                 cells["b"]),
                   "rel_diff_vs_jacobi_max": float(err.max()) if err.size else None,
                   "roofline": roofline("bcs_solve_ilu0 (%d lanes/cell, %d sweeps)" % (
                       iplan.info()["lanes_per_cell"], sw), ims * 1e-3, bytes_launch, iflops, ilds)}
            del iplan, iout
        except bcs.BcsError as e:
            ilu = {"error": str(e)}

    # mass-action rates and Jacobian of the 100k cells assembled on the device
    # (the inputs of the solve), an HBM-streaming kernel
    assemble = None
    if "assemble" in args.forms:
        M = bcs.Mechanism(mech.n, mech.reactants, mech.products, mech.row_ptr, mech.col_idx)
        y = torch.as_tensor(cells["y"], device=dev)
        kk = torch.as_tensor(mech.k, device=dev)
        fo = torch.empty((C, n), dtype=torch.float64, device=dev)
        Jo = torch.empty((C, nnz), dtype=torch.float64, device=dev)

        def asm_step():
            bcs.assemble(M, y, kk, out=(fo, Jo))

        ams_a = timed(asm_step, args.steps)
        same_j = bool(torch.equal(Jo, values))
        abytes = float(C * (8 * n + 8 * n + 8 * nnz) + 8 * mech.R)
        terms = len(mech.term_pos)
        assemble = {"ms_per_step": round(ams_a, 4), "cells_per_s": round(C / (ams_a * 1e-3), 1),
                    "jacobian_equals_generated": same_j,
                    "roofline": roofline("bcs_assemble", ams_a * 1e-3, abytes,
                                         float(C * (3 * terms + 2 * mech.R)), 0.0)}
        del y, kk, fo, Jo, M

    # the Newton systems solved from the cells' concentrations, J assembled
    # inside the solve kernel, against assembling J first and solving it
    mech_solve = None
    if "mech" in args.forms:
        try:
            M = bcs.Mechanism(mech.n, mech.reactants, mech.products, mech.row_ptr, mech.col_idx)
            mplan = bcs.Plan.from_mechanism(M)
            mplan.autotune(values, gamma, b, RTOL, MAXIT)
            y = torch.as_tensor(cells["y"], device=dev)
            kk = torch.as_tensor(mech.k, device=dev)
            Jo = torch.empty((C, nnz), dtype=torch.float64, device=dev)
            mout = [torch.empty_like(o) for o in out[:4]]

            def fused():
                bcs.solve_batch_mech(mplan, y, kk, gamma, b, RTOL, MAXIT, out=mout, workspace=ws)

            def two_step():
                bcs.assemble(M, y, kk, f=False, out=(None, Jo))
                bcs.solve_batch(mplan, Jo, gamma, b, RTOL, MAXIT, out=out, workspace=ws)

            tf = timed(fused, args.steps)
            t2 = timed(two_step, args.steps)
            mst, mres = mout[3].cpu().numpy(), mout[2].cpu().numpy()
            msolved = int(np.sum((mst == 0) & (mres <= RTOL)))
            same = all(bool(torch.equal(a, c)) for a, c in zip(mout, out[:4]))
            mit = mout[1].cpu().numpy().astype(np.float64)
            mech_solve = {
                "value": round(msolved / (tf * 1e-3), 1), "unit": "cells/s", "ms_per_step": round(tf, 4),
                "ms_assemble_then_solve": round(t2, 4), "solved_fraction": round(msolved / C, 5),
                "bitwise_equal_to_assemble_then_solve": same, "lanes_per_cell": mplan.info()["lanes_per_cell"],
                # HBM: y instead of J (8 n instead of 8 nnz bytes read per cell)
                "roofline": roofline("bcs_solve_fp64_mech", tf * 1e-3, float(C * (8 * n + 16 * n + 24)),
                                     float(np.sum(mit * (4 * nnz + 24 * n) + (5 * nnz + 10 * n)) +
                                           C * 3 * len(mech.term_pos)),
                                     float(np.sum(mit * 16 * nnz + 16 * nnz)))}
            del mplan, y, kk, Jo, mout, M
        except bcs.BcsError as e:
            mech_solve = {"error": str(e)}

    # the small configurations: 100 cells (latency) and 10,000 cells (the
    # paper's cell count; its 77 MB fit the Infinity Cache)
    small = {}
    if "small" in args.forms:
        for cfg in (1, 2):
            m1, c1 = config_inputs(cfg)[0]
            V1, G1, B1 = (torch.as_tensor(c1[k], device=dev) for k in ("values", "gamma", "b"))
            p1 = bcs.Plan(m1.row_ptr, m1.col_idx, precond="jacobi")
            p1.autotune(V1, G1, B1, RTOL, MAXIT)
            o1 = [torch.empty((V1.shape[0], m1.n), dtype=torch.float64, device=dev)] + [
                torch.empty(V1.shape[0], dtype=dt, device=dev)
                for dt in (torch.int32, torch.float64, torch.int32, torch.int32)]
            w1 = p1.workspace(V1.shape[0], dev)

            def s1(p1=p1, V1=V1, G1=G1, B1=B1, o1=o1, w1=w1):
                bcs.solve_batch(p1, V1, G1, B1, RTOL, MAXIT, out=o1, workspace=w1)

            reps = 200 if cfg == 1 else args.steps
            t1 = timed(s1, reps)
            st1, rs1, it1 = o1[3].cpu().numpy(), o1[2].cpu().numpy(), o1[1].cpu().numpy()
            sv1 = int(np.sum((st1 == 0) & (rs1 <= RTOL)))
            small["config%d" % cfg] = {
                "ncells": int(V1.shape[0]), "us_per_call": round(t1 * 1e3, 2),
                "value": round(sv1 / (t1 * 1e-3), 1), "unit": "cells/s",
                "solved_fraction": round(sv1 / V1.shape[0], 5), "iters_mean": round(float(it1.mean()), 2),
                "iters_max": int(it1.max()), "lanes_per_cell": p1.info()["lanes_per_cell"]}
            del V1, G1, B1, p1, o1, w1

    peaks = None
    if "peaks" in args.forms:
        from paper_2405_17363_amd.profiling import measure_peaks

        peaks = measure_peaks()
        # the headline's use of each resource against what the probes attain
        roofline_obj["of_attained"] = {
            "hbm": round(roofline_obj["hbm_gbs"] / peaks["hbm_copy_gbs"], 4),
            "alu": round(roofline_obj["valu_tflops"] / peaks["fp64_fma_tflops"], 4),
            "lds": round(roofline_obj["lds_gather_tbs"] / peaks["lds_random_gather_tbs"], 4)}

    cpu = None
    if not args.no_cpu:
        import oracle

        nthreads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
        # pilot on 2000 cells, then a sample sized for about 10 s of CPU work:
        # a prefix of the batch, or the whole batch solved repeatedly
        S0 = min(2000, C)
        t1 = time.perf_counter()
        oracle.solve_batch(mech.row_ptr, mech.col_idx, cells["values"][:S0], cells["gamma"][:S0],
                           cells["b"][:S0], RTOL, MAXIT, precond=1, nthreads=nthreads)
        pilot = time.perf_counter() - t1
        S = int(min(C, max(S0, S0 * 10.0 / max(pilot, 1e-6))))
        reps = max(1, min(20, int(10.0 / max(pilot * S / S0, 1e-6))))
        times = []
        for _ in range(reps):
            t1 = time.perf_counter()
            _, ci_it, ci_res, ci_st = oracle.solve_batch(mech.row_ptr, mech.col_idx, cells["values"][:S],
                                                         cells["gamma"][:S], cells["b"][:S], RTOL, MAXIT,
                                                         precond=1, nthreads=nthreads)
            times.append(time.perf_counter() - t1)
        tcpu = float(np.median(times))
        csolved = int(np.sum((ci_st == 0) & (ci_res <= RTOL)))
        cpu = {"value": round(csolved / tcpu, 1), "unit": "cells/s", "cores": nthreads, "kind": "oracle",
               "sample": f"first {S} of the {C} cells, FP64 BiCGStab + Jacobi, OpenMP static over cells, "
                         f"median of {len(times)} runs of {tcpu:.2f} s",
               "cpu_model": cpu_model()}
        # one thread, on a prefix sized for about 5 s
        S1 = max(200, int(S0 * 5.0 / max(pilot * nthreads, 1e-6)))
        S1 = min(S1, C)
        t1 = time.perf_counter()
        _, c1_it, c1_res, c1_st = oracle.solve_batch(mech.row_ptr, mech.col_idx, cells["values"][:S1],
                                                     cells["gamma"][:S1], cells["b"][:S1], RTOL, MAXIT,
                                                     precond=1, nthreads=1)
        t1 = time.perf_counter() - t1
        cpu["one_thread"] = {"value": round(int(np.sum((c1_st == 0) & (c1_res <= RTOL))) / t1, 1),
                             "unit": "cells/s", "cores": 1, "sample": f"first {S1} cells, one run of {t1:.2f} s"}

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "100k cells, n=80 mass-action mechanism (150 reactions), h in [1e-3,100] s, "
                               "A = I - gamma J, Jacobi, rtol 1e-10, maxit 200",
                   "ncells": C, "n": n, "nnz": nnz, "precision": "fp64", "plan": info},
        "solved_fraction": round(solved / C, 5),
        "iters_mean": round(float(iters.mean()), 2),
        "iters_p99": float(np.percentile(iters, 99)),
        "iters_max": int(iters.max()),
        "status_counts": np.bincount(status, minlength=4).tolist(),
        "unsolved_floor_limited": floor_limited,
        "roofline": roofline_obj,
        "fp32_refine": mixed,
        "fp32_refine_cell_budget": mixed_cell,
        "adjoint": adjoint,
        "multi_mechanism": multi,
        "block_cells_n": block_cells,
        "ilu0": ilu,
        "assemble": assemble,
        "mech_solve": mech_solve,
        "small_configs": small,
        "measured_peaks": peaks,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
