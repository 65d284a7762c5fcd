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
RTOL = 1e-10
MAXIT = 200


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # about 20 ms of untimed work: the GPU's clocks ramp up over the first
    # launches, and shorter warm-ups time the ramp
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--ncells", type=int, default=100_000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32+refine form")
    ap.add_argument("--no-forms", action="store_true", help="skip the adjoint and multi-mechanism timings")
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--cell-order", type=int, default=1, choices=(0, 1),
                    help="1: cells handed out in the cost order (sorted by gamma on the device each step)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy a 1 GiB device buffer (reference for HBM byte counters)")
    return ap.parse_args()


def algorithmic_bytes_per_cell(n: int, nnz: int) -> int:
    # read J values, b, gamma; write x, resid, iters, status (A stays on chip)
    return 8 * nnz + 8 * n + 8 + 8 * n + 8 + 4 + 4


def flops_per_cell(n: int, nnz: int, iters: np.ndarray, status: np.ndarray) -> float:
    # per full iteration: 2 SpMV (2*nnz FMA each) + 6 dots/norms + 4 vector
    # updates = 4 nnz + 24 n; staging (form A, column scaling, ||b||) and the
    # true-residual check = about 3 nnz + 7 n + (2 nnz + 3 n) per confirmation
    it = iters.astype(np.float64)
    return float(np.sum(it * (4 * nnz + 24 * n) + (5 * nnz + 10 * n)))


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
    hbm_gbs = bytes_launch / avg_launch_s / 1e9
    valu_tfs = flops_launch / avg_launch_s / 1e12
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

    fracs = {"hbm": hbm_gbs / HBM_PEAK_GBS, "alu": valu_tfs / FP64_VALU_PEAK}
    # on-chip operand gathers: every stored entry gathers one FP64 operand per
    # SpMV (two per iteration, one for staging's column scaling, one for the
    # true residual)
    lds_bytes = float(np.sum(iters.astype(np.float64) * 16 * nnz + 16 * nnz))
    lds_tbs = lds_bytes / avg_launch_s / 1e12
    bound = max(fracs, key=fracs.get)
    roofline = {
        "bound": bound,
        "achieved": round(hbm_gbs if bound == "hbm" else valu_tfs, 3),
        "peak": HBM_PEAK_GBS if bound == "hbm" else FP64_VALU_PEAK,
        "unit": "GB/s" if bound == "hbm" else "TFLOP/s",
        "frac": round(fracs[bound], 4),
        "traffic": traffic,
        "kernel": "bcs_solve_fp64 (%d lanes/cell, %d rows/lane, %d steps/lane)" % (
            info["lanes_per_cell"], info["rows_per_lane"], info["steps_per_lane"]),
        "avg_launch_ms": round(avg_launch_s * 1e3, 4),
        "hbm_gbs": round(hbm_gbs, 2),
        "hbm_frac": round(fracs["hbm"], 4),
        "fp64_tflops": round(valu_tfs, 3),
        "fp64_frac": round(fracs["alu"], 4),
        "algorithmic_bytes_per_launch": bytes_launch,
        "algorithmic_flops_per_launch": flops_launch,
        "lds_gather_tbs": round(lds_tbs, 2),
        "lds_gather_frac": round(lds_tbs / LDS_PEAK_TBS, 4),
    }

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
            return {"value": round(msolved / (mms * 1e-3), 1), "ms_per_step": round(mms, 4),
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
    if not args.no_mixed:
        mixed = mixed_form("inner")
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
    if not args.no_forms:
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
        del g, xf, res_adj
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
        multi = {"value": round(msolved / (mms * 1e-3), 1), "unit": "cells/s", "ms_per_step": round(mms, 4),
                 "ncells": mc, "solved_fraction": round(msolved / mc, 5),
                 "ms_one_launch_per_mechanism": round(ems, 4),
                 "lanes_per_cell": [pl.info()["lanes_per_cell"] for pl in mplans],
                 "lanes_per_cell_one_launch_per_mechanism": [pl.info()["lanes_per_cell"] for pl in eplans]}
        del MV, MG, MB, res_m
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
                         f"median of {len(times)} runs of {tcpu:.2f} s"}

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
        "roofline": roofline,
        "fp32_refine": mixed,
        "fp32_refine_cell_budget": mixed_cell,
        "adjoint": adjoint,
        "multi_mechanism": multi,
        "block_cells_n": block_cells,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
