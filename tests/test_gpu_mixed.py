"""GPU mixed precision (FP32 inner BiCGStab, FP64 residual and refinement)
against the oracle's FP32/FP64 emulation and dense LU.

Bound for the final x: the same residual-implied bound as FP64
(tests/parity.py), with resid <= rtol required for converged cells.
Statuses agree with the oracle's emulation at least as well as the emulation
agrees with itself when b is perturbed at FP32 rounding level (relative 2^-24
per entry), less one point.  The inner solve runs in FP32, where the GPU and
the emulation differ by FP32 roundings in every operation (fused
multiply-adds, reciprocal-based quotients and the reduction order on the GPU;
separate roundings, IEEE division and sequential sums in the emulation); a
perturbation of one FP64 ulp mostly vanishes in the first cast to FP32 and
would not exercise that sensitivity.  Refinement counts agree within one on
>= 95% of the cells both solve.  Both readings of
the iteration budget are checked: maxit per inner solve (the default) and per
cell over its inner solves.
"""
import numpy as np
import pytest

import oracle
from parity import lu_check, perturb_ulp32
from workload import config_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2405_17363_amd as bcs  # noqa: E402

RTOL = 1e-10


def gpu(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def run_mixed(plan, cells, x0=None, tune=False):
    V, G, B = gpu(cells["values"]), gpu(cells["gamma"]), gpu(cells["b"])
    if tune:
        plan.autotune(V, G, B, RTOL, 200)
    x, it, res, st, ref = bcs.solve_batch(plan, V, G, B, RTOL, 200, x0=None if x0 is None else gpu(x0))
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (x, it, res, st, ref)]


def check_mixed(mech, cells, out, budget, lu_sample, x0=None):
    rp, ci = mech.row_ptr, mech.col_idx
    x, it, res, st, ref = out
    args = (rp, ci, cells["values"], cells["gamma"])
    xo, ito, refo, reso, sto = oracle.mixed_batch(*args, cells["b"], budget=budget, x0=x0)
    _, _, refp, _, stp = oracle.mixed_batch(*args, perturb_ulp32(cells["b"]), budget=budget, x0=x0)
    agree = float(np.mean(st == sto))
    bar = min(0.99, float(np.mean(stp == sto)) - 0.01)
    print(f"budget {budget}: gpu status {np.bincount(st, minlength=4)}, oracle {np.bincount(sto, minlength=4)}, "
          f"agreement {agree:.4f} (bar {bar:.4f}); iters {it.mean():.2f} / {ito.mean():.2f}, refinements "
          f"{ref.mean():.3f} / {refo.mean():.3f}")
    assert agree >= bar
    conv = st == bcs.BCS_CONVERGED
    assert np.all(res[conv] <= RTOL)
    both = conv & (sto == 0)
    assert np.mean(np.abs(ref[both] - refo[both]) <= 1) >= 0.95
    out = lu_check(rp, ci, cells["values"], cells["gamma"], cells["b"], x, res, st, lu_sample)
    print("LU check", out)
    return out, ref


@pytest.mark.parametrize("lanes", [0, 32])
@pytest.mark.parametrize("budget", ["inner", "cell"])
@pytest.mark.parametrize("cfg,nc", [(1, None), (2, 4000)])
def test_mixed_matches_emulation_and_lu(cfg, nc, budget, lanes):
    """lanes 0: the tuner's choice (one cell per wave, the kernel's nested
    loops); 32: two cells per wave (each slot in its own phase)."""
    mech, cells = config_inputs(cfg, ncells=nc)[0]
    plan = bcs.Plan(mech.row_ptr, mech.col_idx, precision="fp32_refine", refine_budget=budget,
                    lanes_per_cell=lanes)
    out = run_mixed(plan, cells)
    C = len(out[3])
    check_mixed(mech, cells, out, budget, np.arange(0, C, max(1, C // 300)))


@pytest.mark.parametrize("budget", ["inner", "cell"])
def test_mixed_config3_full_100k_cells(budget):
    """The mixed form on the benchmark workload at full size (100,000 cells,
    h up to 100 s), as the benchmark runs it (autotuned on the batch, cost
    order on, so slots refill many times and the refinement phases restart on
    new cells): statuses of every cell against the emulation, dense LU on 256
    sampled converged cells of which at least half needed three or more
    refinements."""
    mech, cells = config_inputs(3)[0]
    plan = bcs.Plan(mech.row_ptr, mech.col_idx, precision="fp32_refine", refine_budget=budget)
    out = run_mixed(plan, cells, tune=True)
    x, it, res, st, ref = out
    rng = np.random.default_rng(8)
    conv = np.nonzero(st == 0)[0]
    multi = conv[ref[conv] >= 3]
    sample = np.unique(np.concatenate([rng.choice(multi, min(128, multi.size), replace=False),
                                       rng.choice(conv, 128, replace=False)]))
    assert sample.size >= 250
    res_lu, _ = check_mixed(mech, cells, out, budget, sample)
    assert res_lu["checked"] >= 250


def test_mixed_warm_start():
    mech, cells = config_inputs(2, ncells=2000)[0]
    rp, ci = mech.row_ptr, mech.col_idx
    xl, _ = oracle.lu_batch(rp, ci, cells["values"], cells["gamma"], cells["b"])
    x0 = xl * (1 + 1e-5 * np.random.default_rng(2).standard_normal(xl.shape))
    plan = bcs.Plan(rp, ci, precision="fp32_refine")
    out = run_mixed(plan, cells, x0=x0)
    _, ref = check_mixed(mech, cells, out, "inner", np.arange(0, 2000, 10), x0=x0)
    cold = run_mixed(plan, cells)
    assert out[4].mean() < cold[4].mean()


def test_mixed_edge_cases():
    mech, cells = config_inputs(1, ncells=20)[0]
    vals, b = cells["values"].copy(), cells["b"].copy()
    b[2] = 0.0
    vals[5, 3] = np.nan
    plan = bcs.Plan(mech.row_ptr, mech.col_idx, precision="fp32_refine")
    x, it, res, st, ref = run_mixed(plan, {"values": vals, "gamma": cells["gamma"], "b": b})
    assert st[2] == bcs.BCS_CONVERGED and it[2] == 0 and ref[2] == 0 and np.all(x[2] == 0)
    assert st[5] == bcs.BCS_NONFINITE
    # gamma = 0: A = I, one inner iteration per refinement, FP32 accuracy per step
    x0, it0, res0, st0, ref0 = run_mixed(plan, {"values": cells["values"], "gamma": np.zeros(20), "b": cells["b"]})
    assert np.all(st0 == 0) and np.allclose(x0, cells["b"], rtol=1e-10, atol=0)


def test_mixed_ideal_cells_bitwise_identical():
    mech, cells = config_inputs(2, ncells=2000, mode="ideal")[0]
    plan = bcs.Plan(mech.row_ptr, mech.col_idx, precision="fp32_refine")
    x, it, res, st, ref = run_mixed(plan, cells)
    assert np.all(x == x[0]) and np.all(it == it[0]) and np.all(ref == ref[0])


@pytest.mark.parametrize("lanes", [64, 32])
def test_mixed_cost_order_gives_index_order_results(lanes):
    """Where and when a cell is solved changes nothing in the mixed form
    either: with the cells handed out in the cost order (slots refilled in
    another sequence, the refinement phases restarted on other cells) every
    output is bitwise the index-order output, at one and at two cells per
    wave, for 20,000 cells of the benchmark workload (a cell that ends
    non-finite reports a NaN residual on both sides)."""
    mech, cells = config_inputs(3, ncells=20000)[0]
    outs = []
    for order in (False, True):
        plan = bcs.Plan(mech.row_ptr, mech.col_idx, precision="fp32_refine", lanes_per_cell=lanes,
                        cell_order=order)
        outs.append(run_mixed(plan, cells))
    for a, b in zip(*outs):
        assert np.array_equal(a, b, equal_nan=a.dtype.kind == "f")
