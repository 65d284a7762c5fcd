"""GPU mixed precision (FP32 inner BiCGStab, FP64 residual and refinement)
against the oracle's FP32/FP64 emulation and dense LU.

Bound for the final x: the same residual-implied bound as FP64,
max(1e-8, 4 kappa_2 max(resid, rho_LU)), with resid <= rtol required for
converged cells.  Statuses agree with the oracle's emulation on >= 95% of
cells (refinement in FP32 is sensitive to rounding order near kappa u32 ~ 1);
refinement counts agree within one on >= 90%.
"""
import numpy as np
import pytest

import oracle
from workload import config_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2405_17363_amd as bcs  # noqa: E402

RTOL = 1e-10


def gpu(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def run_mixed(plan, cells):
    x, it, res, st, ref = bcs.solve_batch(plan, gpu(cells["values"]), gpu(cells["gamma"]), gpu(cells["b"]), RTOL,
                                          200)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (x, it, res, st, ref)]


@pytest.mark.parametrize("cfg,nc", [(1, None), (2, 4000), (3, 4000)])
def test_mixed_matches_emulation_and_lu(cfg, nc):
    mech, cells = config_inputs(cfg, ncells=nc)[0]
    rp, ci = mech.row_ptr, mech.col_idx
    plan = bcs.Plan(rp, ci, precision="fp32_refine")
    x, it, res, st, ref = run_mixed(plan, cells)
    xo, ito, refo, reso, sto = oracle.mixed_batch(rp, ci, cells["values"], cells["gamma"], cells["b"])
    print("gpu status", np.bincount(st, minlength=4), "oracle", np.bincount(sto, minlength=4),
          "iters", it.mean(), ito.mean(), "refinements", ref.mean(), refo.mean())
    assert np.mean(st == sto) >= 0.95
    conv = st == bcs.BCS_CONVERGED
    assert np.all(res[conv] <= RTOL)
    both = conv & (sto == 0)
    assert np.mean(np.abs(ref[both] - refo[both]) <= 1) >= 0.90
    sample = np.nonzero(conv)[0][:200]
    xl, _ = oracle.lu_batch(rp, ci, cells["values"][sample], cells["gamma"][sample], cells["b"][sample])
    for q, c in enumerate(sample):
        A = oracle.to_dense(rp, ci, oracle.form_a(rp, ci, cells["values"][c], cells["gamma"][c]))
        kappa = np.linalg.cond(A)
        bn = np.linalg.norm(cells["b"][c])
        rlu = np.linalg.norm(cells["b"][c] - A @ xl[q]) / bn
        err = np.linalg.norm(x[c] - xl[q]) / np.linalg.norm(xl[q])
        assert err <= max(1e-8, 4 * kappa * max(res[c], rlu)), (c, err, kappa)
        rel = np.linalg.norm(cells["b"][c] - A @ x[c]) / bn
        assert rel <= RTOL + 64 * np.finfo(float).eps * np.linalg.norm(np.abs(A) @ np.abs(x[c])) / bn


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
