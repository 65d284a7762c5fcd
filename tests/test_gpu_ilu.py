"""GPU parity of the ILU(0)-preconditioned solve against the CPU oracle.

The oracle's BiCGStab with precond = 2 (ILU(0) by the IKJ elimination on the
pattern, each triangle applied by the same number of Jacobi sweeps) is the
reference: statuses and iteration counts agree at least as well as the oracle
agrees with itself under a one-ulp perturbation of b (less one point; the
GPU evaluates the same operations with FMA and multiplies by the pivots'
reciprocals, a rounding-level difference), and x meets the dense-LU bound of
tests/parity.py.  The pins that need no oracle: gamma = 0 gives x = b in one
iteration (the factors of I are I), and on a tridiagonal pattern, where
ILU(0) is the exact LU factorisation, sweeps at the triangles' depth make the
preconditioner exact, so every cell converges at the first half step.
"""
import numpy as np
import pytest

import oracle
from parity import conservation_check, iters_close, lu_check, perturb_ulp
from workload import config_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - collected on CPU hosts too
    pytest.skip("no GPU", allow_module_level=True)

import paper_2405_17363_amd as bcs  # noqa: E402

RTOL = 1e-10


def gpu(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def run(plan, values, gamma, b, rtol=RTOL, maxit=200, x0=None):
    x, it, res, st, _ = bcs.solve_batch(plan, gpu(values), gpu(np.atleast_1d(gamma)), gpu(b), rtol, maxit,
                                        x0=None if x0 is None else gpu(x0))
    torch.cuda.synchronize()
    return x.cpu().numpy(), it.cpu().numpy(), res.cpu().numpy(), st.cpu().numpy()


def against_oracle(rp, ci, values, gamma, b, it, res, st, sweeps, kind=oracle.J_GAMMA, x0=None, maxit=200):
    args = (rp, ci, values, gamma)
    kw = dict(precond=2, ilu_sweeps=sweeps, kind=kind, x0=x0, maxit=maxit)
    xo, ito, reso, sto = oracle.solve_batch(*args, b, **kw)
    xp, itp, resp, stp = oracle.solve_batch(*args, perturb_ulp(b), **kw)
    bar_agree = min(0.99, float(np.mean(stp == sto)) - 0.01)
    bar_close = min(0.95, iters_close(itp, ito, stp, sto) - 0.01)
    agree = float(np.mean(st == sto))
    close = iters_close(it, ito, st, sto)
    print(f"ILU(0) s={sweeps}: status agreement {agree:.4f} (bar {bar_agree:.4f}), iterations close {close:.4f} "
          f"(bar {bar_close:.4f}); mean iterations GPU {it[st == 0].mean():.2f} oracle {ito[sto == 0].mean():.2f}")
    assert agree >= bar_agree, (np.bincount(st, minlength=4), np.bincount(sto, minlength=4))
    assert close >= bar_close
    assert np.all(res[st == bcs.BCS_CONVERGED] <= RTOL)
    both = (st == 0) & (sto == 0)
    assert abs(it[both].mean() - ito[both].mean()) <= 0.05 * ito[both].mean() + 0.1
    return xo, ito, reso, sto


@pytest.mark.parametrize("sweeps", [1, 2, 3, 4])
@pytest.mark.parametrize("lanes", [0, 32, 64])
def test_config1_against_oracle_and_lu(lanes, sweeps):
    mech, cells = config_inputs(1)[0]
    rp, ci = mech.row_ptr, mech.col_idx
    try:
        plan = bcs.Plan(rp, ci, precond="ilu0", ilu_sweeps=sweeps, lanes_per_cell=lanes)
    except bcs.BcsError as e:
        assert lanes != 0 and e.code == -3, e  # a fixed lane count whose layout does not fit
        pytest.skip(f"no ILU(0) layout at {lanes} lanes: {e}")
    x, it, res, st = run(plan, cells["values"], cells["gamma"], cells["b"])
    print("plan", plan.info())
    against_oracle(rp, ci, cells["values"], cells["gamma"], cells["b"], it, res, st, sweeps)
    out = lu_check(rp, ci, cells["values"], cells["gamma"], cells["b"], x, res, st, np.arange(100))
    assert out["checked"] >= 99


def test_config3_100k_cells_full_size():
    """The benchmark workload at full size with the default sweeps, autotuned on
    the batch as the benchmark runs it: every cell's status and iterations
    against the oracle, conservation on every converged cell, dense LU on 600
    sampled cells plus the 100 stiffest."""
    mech, cells = config_inputs(3)[0]
    rp, ci = mech.row_ptr, mech.col_idx
    plan = bcs.Plan(rp, ci, precond="ilu0")
    V, G, B = gpu(cells["values"]), gpu(cells["gamma"]), gpu(cells["b"])
    plan.autotune(V, G, B, RTOL, 200)
    x, it, res, st, _ = bcs.solve_batch(plan, V, G, B, RTOL, 200)
    torch.cuda.synchronize()
    x, it, res, st = (t.cpu().numpy() for t in (x, it, res, st))
    del V, G, B
    sweeps = plan.options.ilu_sweeps or 3
    print("plan", plan.info(), "status", np.bincount(st, minlength=4))
    assert np.mean(st == bcs.BCS_CONVERGED) >= 0.99
    against_oracle(rp, ci, cells["values"], cells["gamma"], cells["b"], it, res, st, sweeps)
    conservation_check(rp, ci, cells["values"], cells["gamma"], cells["b"], x, st, mech.n)
    rng = np.random.default_rng(3)
    stiff = np.argsort(cells["gamma"])[-100:]
    sample = np.unique(np.concatenate([rng.choice(100_000, 600, replace=False), stiff]))
    out = lu_check(rp, ci, cells["values"], cells["gamma"], cells["b"], x, res, st, sample)
    print("LU check", out)
    assert out["checked"] >= 600


def test_config4_mechanisms():
    for mech, cells in config_inputs(4, ncells=4000):
        rp, ci = mech.row_ptr, mech.col_idx
        try:
            plan = bcs.Plan(rp, ci, precond="ilu0")
        except bcs.BcsError as e:
            # the n = 200 factor block (1878 doubles per slot) may not fit a
            # workgroup's LDS at any lane count
            assert e.code == -3 and mech.n == 200, e
            print("n = 200:", e)
            continue
        x, it, res, st = run(plan, cells["values"], cells["gamma"], cells["b"])
        print("n", mech.n, plan.info(), np.bincount(st, minlength=4))
        against_oracle(rp, ci, cells["values"], cells["gamma"], cells["b"], it, res, st, 3)
        rng = np.random.default_rng(mech.n)
        lu_check(rp, ci, cells["values"], cells["gamma"], cells["b"], x, res, st,
                 rng.choice(len(st), 150, replace=False))


def test_gamma_zero_returns_b_in_one_iteration():
    mech, cells = config_inputs(1)[0]
    plan = bcs.Plan(mech.row_ptr, mech.col_idx, precond="ilu0")
    x, it, res, st = run(plan, cells["values"], np.zeros(100), cells["b"])
    assert np.all(st == 0) and np.all(it == 1)
    assert np.array_equal(x, cells["b"])


@pytest.mark.parametrize("n", [5, 8])
def test_tridiagonal_pattern_exact_factors_converge_at_the_first_half_step(n):
    """No fill: ILU(0) is the LU factorisation; n - 1 sweeps solve each
    triangle exactly (a bidiagonal factor's dependency depth is n - 1)."""
    rp = [0]
    ci = []
    for i in range(n):
        ci += [j for j in (i - 1, i, i + 1) if 0 <= j < n]
        rp.append(len(ci))
    rp, ci = np.array(rp, np.int32), np.array(ci, np.int32)
    rng = np.random.default_rng(n)
    C = 300
    A = rng.standard_normal((C, len(ci)))
    rows = np.repeat(np.arange(n), np.diff(rp))
    A[:, rows == ci] = 4.0 + rng.random((C, n))  # diagonally dominant: no pivoting needed
    b = rng.standard_normal((C, n))
    plan = bcs.Plan(rp, ci, precond="ilu0", ilu_sweeps=n - 1, matrix_kind="a_direct")
    x, it, res, st = run(plan, A, np.zeros(1), b)
    assert np.all(st == 0) and np.all(it == 1), (np.bincount(st), np.bincount(it))
    xl, _ = oracle.lu_batch(rp, ci, A, np.zeros(C), b, kind=oracle.A_DIRECT)
    assert np.max(np.linalg.norm(x - xl, axis=1) / np.linalg.norm(xl, axis=1)) <= 1e-13


def test_a_direct_mode_and_initial_guess():
    mech, cells = config_inputs(2, ncells=3000)[0]
    rp, ci = mech.row_ptr, mech.col_idx
    A = np.stack([oracle.form_a(rp, ci, cells["values"][c], cells["gamma"][c]) for c in range(3000)])
    plan = bcs.Plan(rp, ci, precond="ilu0", matrix_kind="a_direct")
    x, it, res, st = run(plan, A, np.zeros(1), cells["b"])
    against_oracle(rp, ci, A, np.zeros(3000), cells["b"], it, res, st, 3, kind=oracle.A_DIRECT)
    # a warm start halfway to the solution
    x0 = 0.5 * x
    xw, itw, resw, stw = run(plan, A, np.zeros(1), cells["b"], x0=x0)
    against_oracle(rp, ci, A, np.zeros(3000), cells["b"], itw, resw, stw, 3, kind=oracle.A_DIRECT, x0=x0)
    lu_check(rp, ci, A, np.zeros(3000), cells["b"], xw, resw, stw, np.arange(0, 3000, 10), kind=oracle.A_DIRECT)


def test_edge_cases_nan_zero_rhs_maxit():
    mech, cells = config_inputs(1)[0]
    V, g, b = cells["values"].copy(), cells["gamma"].copy(), cells["b"].copy()
    V[3, 5] = np.nan
    b[7] = 0.0
    plan = bcs.Plan(mech.row_ptr, mech.col_idx, precond="ilu0")
    x, it, res, st = run(plan, V, g, b)
    assert st[3] == bcs.BCS_NONFINITE
    assert st[7] == bcs.BCS_CONVERGED and it[7] == 0 and np.all(x[7] == 0) and res[7] == 0
    assert np.all(np.isfinite(x[np.arange(100) != 3]))
    x1, it1, res1, st1 = run(plan, V, g, b, maxit=1)
    assert np.all(it1 <= 1)
    against_oracle(mech.row_ptr, mech.col_idx, V, g, b, it1, res1, st1, 3, maxit=1)


def test_permutation_and_repetition_bitwise():
    mech, cells = config_inputs(2, ncells=4000)[0]
    plan = bcs.Plan(mech.row_ptr, mech.col_idx, precond="ilu0")
    out1 = run(plan, cells["values"], cells["gamma"], cells["b"])
    out2 = run(plan, cells["values"], cells["gamma"], cells["b"])
    perm = np.random.default_rng(5).permutation(4000)
    outp = run(plan, cells["values"][perm], cells["gamma"][perm], cells["b"][perm])
    for a, b2, c in zip(out1, out2, outp):
        assert np.array_equal(a, b2)
        assert np.array_equal(a[perm], c)


def test_ilu_plans_reject_the_adjoint_and_the_one_launch_form():
    mech, cells = config_inputs(1)[0]
    plan = bcs.Plan(mech.row_ptr, mech.col_idx, precond="ilu0")
    V, G, B = gpu(cells["values"]), gpu(cells["gamma"]), gpu(cells["b"])
    x, _, _, _, _ = bcs.solve_batch(plan, V, G, B)
    with pytest.raises(bcs.BcsError) as e:
        bcs.solve_batch_adjoint(plan, V, G, x, B)
    assert e.value.code == -3
    with pytest.raises(bcs.BcsError) as e:
        bcs.solve_multi([plan], [V], [G], [B])
    assert e.value.code == -3
