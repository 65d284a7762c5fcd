"""GPU parity: the HIP batched BiCGStab (through the C-ABI) against the CPU oracle.

x is compared with the oracle's dense LU under the bound the residual implies
(tests/parity.py: flat 1e-8 norm-wise plus a component-wise bound where
kappa_2 * max(resid, rho_LU) <= 1e-8, else 4 kappa_2 max(resid, rho_LU)),
statuses and iteration counts (within max(3, 15%)) with the oracle's
BiCGStab at least as well as the oracle agrees with itself under a one-ulp
perturbation of b, less one point (BiCGStab's iteration count is rounding
sensitive; beyond that it is parity unpinned).  Bitwise properties (ideal
cells, permutations, repeated runs, lanes/slot independence) are exact.
"""
import numpy as np
import pytest

import oracle
from parity import conservation_check, iters_close, lu_check, perturb_ulp
from workload import config_inputs, gen_cells, gen_mechanism

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - collected on CPU hosts too
    pytest.skip("no GPU", allow_module_level=True)

import paper_2405_17363_amd as bcs  # noqa: E402

RTOL = 1e-10


def gpu(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def run(plan, values, gamma, b, rtol=RTOL, maxit=200, x0=None):
    x, it, res, st, ref = bcs.solve_batch(plan, gpu(values), gpu(np.atleast_1d(gamma)), gpu(b), rtol, maxit,
                                          x0=None if x0 is None else gpu(x0))
    torch.cuda.synchronize()
    return x.cpu().numpy(), it.cpu().numpy(), res.cpu().numpy(), st.cpu().numpy()


def check_against_lu(rp, ci, values, gamma, b, x, res, st, sample, kind=oracle.J_GAMMA):
    out = lu_check(rp, ci, values, gamma, b, x, res, st, sample, kind=kind)
    print("LU check", out)
    return out


def check_against_oracle(mech, cells, x, it, res, st, precond=1, control=True, x0=None):
    """Statuses and iteration counts against the oracle, at least as close as the
    oracle to itself under a one-ulp perturbation of b (less one point)."""
    args = (mech.row_ptr, mech.col_idx, cells["values"], cells["gamma"])
    xo, ito, reso, sto = oracle.solve_batch(*args, cells["b"], precond=precond, x0=x0)
    agree = float(np.mean(st == sto))
    close = iters_close(it, ito, st, sto)
    ref_agree, ref_close = 0.99, 0.95
    if control:
        xp, itp, resp, stp = oracle.solve_batch(*args, perturb_ulp(cells["b"]), precond=precond, x0=x0)
        ref_agree = min(ref_agree, float(np.mean(stp == sto)) - 0.01)
        ref_close = min(ref_close, iters_close(itp, ito, stp, sto) - 0.01)
    print(f"status agreement {agree:.4f} (bar {ref_agree:.4f}), iterations close {close:.4f} (bar {ref_close:.4f})")
    assert agree >= ref_agree, (agree, ref_agree, np.bincount(st, minlength=4), np.bincount(sto, minlength=4))
    assert np.all(res[st == bcs.BCS_CONVERGED] <= RTOL)
    assert close >= ref_close, (close, ref_close)
    return xo, ito, reso, sto


# ---------------------------------------------------------------- configs ----

@pytest.mark.parametrize("jit", [True, False])
@pytest.mark.parametrize("lanes", [0, 16, 32, 64])
def test_config1_100_cells_all_lane_layouts(lanes, jit):
    mech, cells = config_inputs(1)[0]
    plan = bcs.Plan(mech.row_ptr, mech.col_idx, lanes_per_cell=lanes, jit=jit)
    x, it, res, st = run(plan, cells["values"], cells["gamma"], cells["b"])
    print("plan", plan.info(), "status", np.bincount(st, minlength=4), "iters mean", it.mean())
    check_against_oracle(mech, cells, x, it, res, st)
    check_against_lu(mech.row_ptr, mech.col_idx, cells["values"], cells["gamma"], cells["b"], x, res, st,
                     np.arange(100))


def test_config2_10k_cells_every_cell_against_lu():
    mech, cells = config_inputs(2)[0]
    plan = bcs.Plan(mech.row_ptr, mech.col_idx)
    x, it, res, st = run(plan, cells["values"], cells["gamma"], cells["b"])
    check_against_oracle(mech, cells, x, it, res, st)
    out = check_against_lu(mech.row_ptr, mech.col_idx, cells["values"], cells["gamma"], cells["b"], x, res, st,
                           np.arange(10_000))
    assert out["checked"] >= 9900
    assert np.mean(st == bcs.BCS_CONVERGED) >= 0.99
    conservation_check(mech.row_ptr, mech.col_idx, cells["values"], cells["gamma"], cells["b"], x, st, mech.n)


def test_config3_100k_cells_full_size():
    """The benchmark workload at full size, in the launch configuration the
    benchmark times (autotuned on the batch, cost order on): statuses and
    iterations of every cell against the oracle, conservation on every
    converged cell, dense LU on 600 sampled cells plus the 100 stiffest."""
    mech, cells = config_inputs(3)[0]
    plan = bcs.Plan(mech.row_ptr, mech.col_idx)
    V, G, B = gpu(cells["values"]), gpu(cells["gamma"]), gpu(cells["b"])
    plan.autotune(V, G, B, RTOL, 200)
    x, it, res, st, _ = bcs.solve_batch(plan, V, G, B, RTOL, 200)
    torch.cuda.synchronize()
    x, it, res, st = (t.cpu().numpy() for t in (x, it, res, st))
    del V, G, B
    conv = st == bcs.BCS_CONVERGED
    assert conv.mean() >= 0.99
    check_against_oracle(mech, cells, x, it, res, st)
    conservation_check(mech.row_ptr, mech.col_idx, cells["values"], cells["gamma"], cells["b"], x, st, mech.n)
    rng = np.random.default_rng(3)
    stiff = np.argsort(cells["gamma"])[-100:]
    sample = np.unique(np.concatenate([rng.choice(100_000, 600, replace=False), stiff]))
    out = check_against_lu(mech.row_ptr, mech.col_idx, cells["values"], cells["gamma"], cells["b"], x, res, st,
                           sample)
    assert out["checked"] >= 600


def test_config4_three_mechanisms_separately():
    for mech, cells in config_inputs(4, ncells=8000):
        plan = bcs.Plan(mech.row_ptr, mech.col_idx)
        x, it, res, st = run(plan, cells["values"], cells["gamma"], cells["b"])
        print("n", mech.n, plan.info(), np.bincount(st, minlength=4))
        check_against_oracle(mech, cells, x, it, res, st)
        rng = np.random.default_rng(mech.n)
        check_against_lu(mech.row_ptr, mech.col_idx, cells["values"], cells["gamma"], cells["b"], x, res, st,
                         rng.choice(len(st), 120, replace=False))


def test_precond_none_matches_oracle():
    mech, cells = config_inputs(1)[0]
    plan = bcs.Plan(mech.row_ptr, mech.col_idx, precond="none")
    x, it, res, st = run(plan, cells["values"], cells["gamma"], cells["b"])
    check_against_oracle(mech, cells, x, it, res, st, precond=0)
    check_against_lu(mech.row_ptr, mech.col_idx, cells["values"], cells["gamma"], cells["b"], x, res, st,
                     np.arange(100))


# ------------------------------------------------------- small systems -------

def _csr_dense(M):
    n = M.shape[0]
    rp, ci, vals = [0], [], []
    for i in range(n):
        for j in range(n):
            if M[i, j] != 0 or i == j:
                ci.append(j)
                vals.append(M[i, j])
        rp.append(len(ci))
    return np.array(rp, np.int32), np.array(ci, np.int32), np.array(vals)


@pytest.mark.parametrize("jit", [True, False])
@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_tiny_random_systems_vs_lu(precond, jit):
    rng = np.random.default_rng(11)
    for trial in range(40):
        n = int(rng.integers(1, 13))
        M = np.where(rng.uniform(size=(n, n)) < 0.5, rng.standard_normal((n, n)), 0.0)
        M[np.arange(n), np.arange(n)] = rng.uniform(1, 3, n) * rng.choice([-1, 1], n)
        rp, ci, vals = _csr_dense(M)
        C = 37  # several cells of the same pattern, different values
        V = vals[None, :] * rng.uniform(0.5, 1.5, (C, vals.size))
        b = rng.standard_normal((C, n))
        plan = bcs.Plan(rp, ci, precond=precond, matrix_kind="a_direct", jit=jit)
        x, it, res, st = run(plan, V, [0.0], b, rtol=1e-12, maxit=400)
        xo, ito, reso, sto = oracle.solve_batch(rp, ci, V, [0.0], b, rtol=1e-12, maxit=400,
                                                precond=int(precond == "jacobi"), kind=oracle.A_DIRECT)
        for c in range(C):
            A = oracle.to_dense(rp, ci, V[c])
            if np.linalg.cond(A) > 1e6 or sto[c] == oracle.BREAKDOWN:
                continue
            assert st[c] == bcs.BCS_CONVERGED, (trial, c, st[c], it[c], res[c])
            xr = np.linalg.solve(A, b[c])
            assert np.linalg.norm(x[c] - xr) <= 4 * np.linalg.cond(A) * max(res[c], 1e-15) * np.linalg.norm(xr) \
                + 1e-13


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_finite_termination_on_gpu(k):
    # SPD with k distinct eigenvalues: BiCGStab stops within k iterations
    rng = np.random.default_rng(k)
    n = 12
    eigs = np.array([1.0, 2.5, 4.0, 6.0][:k])
    C = 16
    Ms = []
    for c in range(C):
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        Ms.append(Q @ np.diag(eigs[np.arange(n) % k]) @ Q.T)
    rp, ci, _ = _csr_dense(np.ones((n, n)))
    V = np.stack([M.reshape(-1) for M in Ms])
    b = rng.standard_normal((C, n))
    plan = bcs.Plan(rp, ci, precond="none", matrix_kind="a_direct")
    x, it, res, st = run(plan, V, [0.0], b, rtol=1e-9, maxit=50)
    assert np.all(st == bcs.BCS_CONVERGED) and np.all(it <= k), it


# ----------------------------------------------------- closed forms / edges --

def test_gamma_zero_returns_b_in_one_iteration():
    mech, cells = config_inputs(1, ncells=64)[0]
    plan = bcs.Plan(mech.row_ptr, mech.col_idx)
    x, it, res, st = run(plan, cells["values"], np.zeros(64), cells["b"])
    assert np.all(st == 0) and np.all(it == 1) and np.array_equal(x, cells["b"]) and np.all(res == 0)


def test_scalar_gamma_equals_broadcast_gamma():
    mech, cells = config_inputs(1, ncells=50)[0]
    plan = bcs.Plan(mech.row_ptr, mech.col_idx)
    a = run(plan, cells["values"], [0.3], cells["b"])
    b = run(plan, cells["values"], np.full(50, 0.3), cells["b"])
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_diagonal_system_with_jacobi():
    n = 40
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    rng = np.random.default_rng(5)
    d = rng.uniform(1, 1e4, (9, n))
    b = rng.standard_normal((9, n))
    plan = bcs.Plan(rp, ci, matrix_kind="a_direct")
    x, it, res, st = run(plan, d, [0.0], b)
    assert np.all(st == 0) and np.all(it == 1)
    # x = (1/d) * (alpha * b) with alpha = (b.b)/(b.Ahat b), Ahat = A D^-1: four roundings
    assert np.allclose(x, b / d, rtol=2e-15, atol=0)


def test_edge_cases_nan_zero_rhs_maxit():
    mech, cells = config_inputs(1, ncells=40)[0]
    plan = bcs.Plan(mech.row_ptr, mech.col_idx)
    vals, b = cells["values"].copy(), cells["b"].copy()
    vals[3, 7] = np.nan
    b[5] = 0.0
    b[9, 2] = np.inf
    x, it, res, st = run(plan, vals, cells["gamma"], b)
    assert st[3] == bcs.BCS_NONFINITE and st[9] == bcs.BCS_NONFINITE
    assert st[5] == bcs.BCS_CONVERGED and it[5] == 0 and res[5] == 0 and np.all(x[5] == 0)
    clean = run(plan, cells["values"], cells["gamma"], cells["b"])
    keep = [c for c in range(40) if c not in (3, 5, 9)]
    for u, v in zip((x, it, res, st), clean):
        assert np.array_equal(u[keep], v[keep])
    x1, it1, res1, st1 = run(plan, cells["values"], cells["gamma"], cells["b"], maxit=1)
    assert np.all(it1 == 1) and np.all((st1 == bcs.BCS_MAXIT) | (st1 == bcs.BCS_CONVERGED))


def test_exact_breakdown_and_singular_cells():
    rp = np.array([0, 2, 4], np.int32)
    ci = np.array([0, 1, 0, 1], np.int32)
    A = np.array([[0.0, 1.0, -1.0, 0.0]])
    plan = bcs.Plan(rp, ci, precond="none", matrix_kind="a_direct")
    x, it, res, st = run(plan, A, [0.0], np.array([[1.0, 0.0]]))
    assert st[0] == bcs.BCS_BREAKDOWN and it[0] == 2 and np.all(x[0] == 0) and res[0] == 1.0
    # J mode, diagonal pattern, A = I - g J = 0
    n, g = 4, 0.5
    rpd = np.arange(n + 1, dtype=np.int32)
    cid = np.arange(n, dtype=np.int32)
    J = np.full((1, n), 1.0 / g)
    x, it, res, st = run(bcs.Plan(rpd, cid, precond="none"), J, [g], np.ones((1, n)))
    assert st[0] == bcs.BCS_BREAKDOWN
    x, it, res, st = run(bcs.Plan(rpd, cid, precond="jacobi"), J, [g], np.ones((1, n)))
    assert st[0] == bcs.BCS_NONFINITE


def test_largest_supported_n():
    """n = 255, the largest cell (8-bit gather indices; index 255 is the zero
    spare element): only 64 lanes per cell fit its registers."""
    mech = gen_mechanism(255, 510)
    cells = gen_cells(mech, 300, seed=255, h_max=10.0)
    plan = bcs.Plan(mech.row_ptr, mech.col_idx)
    assert plan.info()["lanes_per_cell"] == 64
    x, it, res, st = run(plan, cells["values"], cells["gamma"], cells["b"])
    check_against_oracle(mech, cells, x, it, res, st)
    sample = np.random.default_rng(3).choice(300, 30, replace=False)
    check_against_lu(mech.row_ptr, mech.col_idx, cells["values"], cells["gamma"], cells["b"], x, res, st, sample)


def test_pattern_no_layout_holds_is_rejected():
    """A dense 200-entry row needs more schedule steps than any lane count's
    registers hold: plan creation fails with an error, nothing is launched."""
    n = 200
    rows = [list(range(n))] + [[i] for i in range(1, n)]
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    ci = np.concatenate(rows).astype(np.int32)
    with pytest.raises(bcs.BcsError, match="no kernel layout"):
        bcs.Plan(rp, ci)


def test_zero_cells_is_a_noop():
    mech = gen_mechanism(30, 50)
    plan = bcs.Plan(mech.row_ptr, mech.col_idx)
    x, it, res, st = run(plan, np.zeros((0, mech.nnz)), [0.1], np.zeros((0, mech.n)))
    assert x.shape == (0, mech.n)


# ------------------------------------------------------ bitwise properties ---

def test_ideal_cells_bitwise_identical_and_slot_independent():
    mech, cells = config_inputs(2, ncells=3000, mode="ideal")[0]
    plan = bcs.Plan(mech.row_ptr, mech.col_idx)
    x, it, res, st = run(plan, cells["values"], cells["gamma"], cells["b"])
    assert np.all(x == x[0]) and np.all(it == it[0]) and np.all(res == res[0]) and np.all(st == st[0])


@pytest.mark.parametrize("jit", [True, False])
def test_permutation_and_repetition_bitwise(jit):
    mech, cells = config_inputs(2, ncells=5000)[0]
    plan = bcs.Plan(mech.row_ptr, mech.col_idx, jit=jit)
    a = run(plan, cells["values"], cells["gamma"], cells["b"])
    a2 = run(plan, cells["values"], cells["gamma"], cells["b"])
    perm = np.random.default_rng(9).permutation(5000)
    p = run(plan, cells["values"][perm], cells["gamma"][perm], cells["b"][perm])
    for u, v, w in zip(a, a2, p):
        assert np.array_equal(u, v)
        assert np.array_equal(u[perm], w)


# ------------------------------------------- one launch, several mechanisms --

def test_config4_single_persistent_launch_full_size():
    """Config 4 at its full 50,000 cells (12,500 / 25,000 / 12,500 over n = 30,
    80, 200), in the launch configuration the benchmark times (lanes chosen by
    the one-launch autotuner): every cell bitwise equal to its own
    mechanism's launch, statuses and iterations of every cell against the
    oracle, dense LU on sampled cells."""
    mechs = config_inputs(4)
    plans = [bcs.Plan(m.row_ptr, m.col_idx) for m, _ in mechs]
    V = [gpu(c["values"]) for _, c in mechs]
    Gm = [gpu(c["gamma"]) for _, c in mechs]
    Bv = [gpu(c["b"]) for _, c in mechs]
    assert sum(v.shape[0] for v in V) == 50_000
    bcs.multi_autotune(plans, V, Gm, Bv, RTOL, 200)
    outs = bcs.solve_multi(plans, V, Gm, Bv, RTOL, 200)
    torch.cuda.synchronize()
    for (mech, cells), plan, (x, it, res, st), v, g, b in zip(mechs, plans, outs, V, Gm, Bv):
        x, it, res, st = (t.cpu().numpy() for t in (x, it, res, st))
        # the same per-cell arithmetic as the single-mechanism kernel
        xs, its, ress, sts, _ = bcs.solve_batch(plan, v, g, b, RTOL, 200)
        torch.cuda.synchronize()
        assert np.array_equal(st, sts.cpu().numpy()) and np.array_equal(it, its.cpu().numpy())
        assert np.array_equal(x, xs.cpu().numpy()) and np.array_equal(res, ress.cpu().numpy())
        check_against_oracle(mech, cells, x, it, res, st)
        rng = np.random.default_rng(mech.n + 1)
        check_against_lu(mech.row_ptr, mech.col_idx, cells["values"], cells["gamma"], cells["b"], x, res, st,
                         rng.choice(len(st), 200, replace=False))


def test_multi_rejects_bad_arguments_and_accepts_empty_mechanisms():
    mechs = config_inputs(4, ncells=400)
    plans = [bcs.Plan(m.row_ptr, m.col_idx) for m, _ in mechs]
    V = [gpu(c["values"]) for _, c in mechs]
    Gm = [gpu(c["gamma"]) for _, c in mechs]
    Bv = [gpu(c["b"]) for _, c in mechs]
    with pytest.raises(bcs.BcsError):
        bcs.solve_multi([plans[0], plans[0]], V[:1] * 2, Gm[:1] * 2, Bv[:1] * 2)
    empty = [gpu(np.zeros((0, plans[1].nnz))), gpu(np.zeros(1)), gpu(np.zeros((0, plans[1].n)))]
    outs = bcs.solve_multi([plans[0], plans[1]], [V[0], empty[0]], [Gm[0], empty[1]], [Bv[0], empty[2]])
    torch.cuda.synchronize()
    assert outs[1][0].shape[0] == 0
    xs, its, ress, sts, _ = bcs.solve_batch(plans[0], V[0], Gm[0], Bv[0])
    torch.cuda.synchronize()
    assert torch.equal(outs[0][0], xs) and torch.equal(outs[0][3], sts)
    # the one-launch autotuner leaves a mechanism without cells as it is
    before = plans[1].info()["lanes_per_cell"]
    lanes = bcs.multi_autotune([plans[0], plans[1]], [V[0], empty[0]], [Gm[0], empty[1]], [Bv[0], empty[2]])
    assert lanes[1] == before and lanes[0] in (16, 32, 64)
    with pytest.raises(bcs.BcsError):
        bcs.multi_autotune([plans[0], plans[0]], V[:1] * 2, Gm[:1] * 2, Bv[:1] * 2)


def test_multi_autotune_keeps_results_and_fixed_lanes():
    """The one-launch autotuner only changes lane counts: afterwards each
    mechanism's part of the combined launch still equals its own launch with
    the chosen kernel, the adjoint kernels follow the choice, and a plan whose
    lanes the caller fixed keeps them."""
    mechs = config_inputs(4, ncells=6000)
    m0 = mechs[0][0]  # n = 30, fixed at 32 lanes per cell
    plans = [bcs.Plan(m0.row_ptr, m0.col_idx, lanes_per_cell=32)]
    plans += [bcs.Plan(m.row_ptr, m.col_idx) for m, _ in mechs[1:]]
    V = [gpu(c["values"]) for _, c in mechs]
    Gm = [gpu(c["gamma"]) for _, c in mechs]
    Bv = [gpu(c["b"]) for _, c in mechs]
    lanes = bcs.multi_autotune(plans, V, Gm, Bv, RTOL, 200)
    assert len(lanes) == len(plans) and all(L in (16, 32, 64) for L in lanes) and lanes[0] == 32
    assert [p.info()["lanes_per_cell"] for p in plans] == lanes
    outs = bcs.solve_multi(plans, V, Gm, Bv, RTOL, 200)
    torch.cuda.synchronize()
    for (mech, cells), plan, (x, it, res, st), v, g, b in zip(mechs, plans, outs, V, Gm, Bv):
        xs, its, ress, sts, _ = bcs.solve_batch(plan, v, g, b, RTOL, 200)
        torch.cuda.synchronize()
        assert torch.equal(x, xs) and torch.equal(it, its) and torch.equal(res, ress) and torch.equal(st, sts)
        check_against_oracle(mech, cells, *(t.cpu().numpy() for t in (x, it, res, st)))
        gb = torch.ones_like(b)
        ast = bcs.solve_batch_adjoint(plan, v, g, xs, gb, RTOL, 200)[5]
        torch.cuda.synchronize()
        assert float((ast == 0).double().mean()) > 0.95


@pytest.mark.parametrize("lanes", [16, 32, 64])
def test_schedule_shapes_against_plain_schedule(lanes, monkeypatch):
    """The specialised kernels' schedules leave the diagonal out (its term
    starts each row sum) and let the longest rows span two slots.  Both the
    shaped and the plain schedule (BCS_SCHED=0) must meet the oracle and LU
    bar on config 2, and the shaped one must be shorter."""
    mech, cells = config_inputs(2, ncells=4000)[0]
    monkeypatch.setenv("BCS_SCHED", "0")
    plain = bcs.Plan(mech.row_ptr, mech.col_idx, lanes_per_cell=lanes)
    monkeypatch.delenv("BCS_SCHED")
    shaped = bcs.Plan(mech.row_ptr, mech.col_idx, lanes_per_cell=lanes)
    assert shaped.info()["steps_per_lane"] < plain.info()["steps_per_lane"]
    sample = np.random.default_rng(lanes).choice(4000, 60, replace=False)
    for plan in (plain, shaped):
        x, it, res, st = run(plan, cells["values"], cells["gamma"], cells["b"])
        check_against_oracle(mech, cells, x, it, res, st)
        check_against_lu(mech.row_ptr, mech.col_idx, cells["values"], cells["gamma"], cells["b"], x, res, st, sample)


def test_cost_order_gives_index_order_results():
    """Handing cells out sorted by gamma changes only where and when a cell is
    solved: every output is bitwise the index-order output, every cell is
    written (outputs start as NaN), also for a second, smaller batch that
    reuses the plan's order array (9,001 cells: more than the 8,192 cell
    slots even four resident 32-lane workgroups per CU give), for a batch of
    100 cells (fewer cells than slots: no sort, one cell per slot), and for
    the adjoint."""
    mech, cells = config_inputs(2)[0]
    V, G, B = gpu(cells["values"]), gpu(cells["gamma"]), gpu(cells["b"])
    p0 = bcs.Plan(mech.row_ptr, mech.col_idx, lanes_per_cell=32, cell_order=False)
    p1 = bcs.Plan(mech.row_ptr, mech.col_idx, lanes_per_cell=32, cell_order=True)
    for C in (V.shape[0], 9001, 100):
        ref = bcs.solve_batch(p0, V[:C], G[:C], B[:C], RTOL, 200)
        out = [torch.full((C, mech.n), float("nan"), dtype=torch.float64, device="cuda"),
               torch.full((C,), -1, dtype=torch.int32, device="cuda"),
               torch.full((C,), float("nan"), dtype=torch.float64, device="cuda"),
               torch.full((C,), -1, dtype=torch.int32, device="cuda"),
               torch.full((C,), -1, dtype=torch.int32, device="cuda")]
        got = bcs.solve_batch(p1, V[:C], G[:C], B[:C], RTOL, 200, out=out)
        torch.cuda.synchronize()
        for a, b in zip(ref[:4], got[:4]):
            assert torch.equal(a, b)
    W = gpu(np.random.default_rng(3).standard_normal((V.shape[0], mech.n)))
    x = bcs.solve_batch(p0, V, G, B, RTOL, 200)[0]
    a0 = bcs.solve_batch_adjoint(p0, V, G, x, W, RTOL, 200, grad_gamma=True)
    a1 = bcs.solve_batch_adjoint(p1, V, G, x, W, RTOL, 200, grad_gamma=True)
    torch.cuda.synchronize()
    for a, b in zip(a0, a1):
        assert torch.equal(a, b)


def test_multi_rejects_layouts_beyond_64_kib_before_anything_runs():
    """The one-launch form keeps every mechanism's schedule tables in LDS and
    gathers through 16-bit addresses: a combination whose layout exceeds 64 KiB
    is rejected with BCS_ERR_UNSUPPORTED before anything is compiled or
    launched (the outputs stay untouched)."""
    mech = gen_mechanism(200, 400)
    # eight plans of the n = 200 mechanism at 64 lanes per cell: the tables
    # alone (steps x 64 lanes x 4 bytes + 4 n bytes each) exceed 64 KiB
    d = bcs.schedule_describe(mech.row_ptr, mech.col_idx, 64)
    assert 8 * (d["steps"] * 64 * 4 + 4 * mech.n) > 65536
    plans = [bcs.Plan(mech.row_ptr, mech.col_idx, lanes_per_cell=64, autotune=False) for _ in range(8)]
    cells = gen_cells(mech, 16, seed=7)
    V, G, B = gpu(cells["values"]), gpu(cells["gamma"]), gpu(cells["b"])
    m = len(plans)
    outs_before = torch.full((16, mech.n), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(bcs.BcsError) as e:
        bcs.solve_multi(plans, [V] * m, [G] * m, [B] * m, RTOL, 200)
    assert e.value.code == -3 and "LDS" in str(e.value)
    torch.cuda.synchronize()
    assert torch.all(outs_before == 7.0)


# ------------------------------------------------------------ initial guess --

def test_initial_guess_at_the_lu_solution_returns_it_without_iterating():
    mech, cells = config_inputs(2, ncells=2000)[0]
    rp, ci = mech.row_ptr, mech.col_idx
    xl, _ = oracle.lu_batch(rp, ci, cells["values"], cells["gamma"], cells["b"])
    plan = bcs.Plan(rp, ci)
    x, it, res, st = run(plan, cells["values"], cells["gamma"], cells["b"], x0=xl)
    xo, ito, reso, sto = oracle.solve_batch(rp, ci, cells["values"], cells["gamma"], cells["b"], precond=1, x0=xl)
    zero = ito == 0
    assert zero.mean() > 0.5
    # cells the oracle finishes without iterating: returned as given, 0 iterations
    agree = (it[zero] == 0) & np.all(x[zero] == xl[zero], axis=1)
    assert agree.mean() >= 0.99, agree.mean()
    check_against_lu(rp, ci, cells["values"], cells["gamma"], cells["b"], x, res, st, np.arange(2000))


def test_warm_start_matches_the_oracle_and_saves_iterations():
    """x0 = a perturbed solution (a Newton-like warm start): statuses and
    iterations against the oracle started from the same x0, x against LU, and
    fewer iterations than a cold start.  x0 may be the output array itself."""
    mech, cells = config_inputs(2, ncells=4000)[0]
    rp, ci = mech.row_ptr, mech.col_idx
    xl, _ = oracle.lu_batch(rp, ci, cells["values"], cells["gamma"], cells["b"])
    x0 = xl * (1 + 1e-4 * np.random.default_rng(5).standard_normal(xl.shape))
    plan = bcs.Plan(rp, ci)
    x, it, res, st = run(plan, cells["values"], cells["gamma"], cells["b"], x0=x0)
    check_against_oracle(mech, cells, x, it, res, st, x0=x0)
    check_against_lu(rp, ci, cells["values"], cells["gamma"], cells["b"], x, res, st, np.arange(0, 4000, 7))
    _, it_cold, _, _ = run(plan, cells["values"], cells["gamma"], cells["b"])
    # a relative 1e-4 error in x0 leaves about six of the ten digits to gain,
    # so the warm start saves iterations, by how many the oracle decides (above)
    assert it.mean() < it_cold.mean()
    # in place: the output array holds x0 on entry
    V, G, B = gpu(cells["values"]), gpu(cells["gamma"]), gpu(cells["b"])
    xin = gpu(x0)
    out = [xin, torch.empty(4000, dtype=torch.int32, device="cuda"),
           torch.empty(4000, dtype=torch.float64, device="cuda"), torch.empty(4000, dtype=torch.int32, device="cuda"),
           None]
    bcs.solve_batch(plan, V, G, B, RTOL, 200, out=out, x0=xin)
    torch.cuda.synchronize()
    assert np.array_equal(xin.cpu().numpy(), x)


@pytest.mark.parametrize("form", ["fp64", "fp64_small", "adjoint", "adjoint_small", "mixed", "mixed_small", "ilu0",
                                  "ilu0_small"])
def test_work_queue_hands_every_cell_out_exactly_once(form, monkeypatch):
    """Debug counter (bcs_debug_count_visits, compiled in with
    BCS_DEBUG_VISITS): on the 100k-cell workload, in the cost order, every
    cell's outputs are written exactly once, and the outputs (pre-filled
    with sentinels) are all written.  The _small forms: 1,000 of the cells,
    no more than the launch's slots, so slot k solves cell k with no queue."""
    monkeypatch.setenv("BCS_DEBUG_VISITS", "1")
    mech, cells = config_inputs(3)[0]
    if form.endswith("_small"):
        cells = {k: v[:1000] for k, v in cells.items()}
        form = form[:-len("_small")]
    C = cells["b"].shape[0]
    kw = {"fp64": {}, "adjoint": {}, "mixed": {"precision": "fp32_refine"}, "ilu0": {"precond": "ilu0"}}[form]
    plan = bcs.Plan(mech.row_ptr, mech.col_idx, **kw)
    V, G, B = gpu(cells["values"]), gpu(cells["gamma"]), gpu(cells["b"])
    counts = torch.zeros(C, dtype=torch.int32, device="cuda")
    L = bcs.lib()
    if form == "adjoint":
        x, _, _, _, _ = bcs.solve_batch(plan, V, G, B, RTOL, 200)
        torch.cuda.synchronize()
        L.bcs_debug_count_visits(counts.data_ptr())
        try:
            _, _, _, it, res, st = bcs.solve_batch_adjoint(plan, V, G, x, B, RTOL, 200)
            torch.cuda.synchronize()
        finally:
            L.bcs_debug_count_visits(None)
    else:
        out = (torch.full((C, mech.n), np.nan, dtype=torch.float64, device="cuda"),
               torch.full((C,), -7, dtype=torch.int32, device="cuda"),
               torch.full((C,), np.nan, dtype=torch.float64, device="cuda"),
               torch.full((C,), -7, dtype=torch.int32, device="cuda"),
               torch.full((C,), -7, dtype=torch.int32, device="cuda"))
        L.bcs_debug_count_visits(counts.data_ptr())
        try:
            _, it, res, st, _ = bcs.solve_batch(plan, V, G, B, RTOL, 200, out=out)
            torch.cuda.synchronize()
        finally:
            L.bcs_debug_count_visits(None)
    c = counts.cpu().numpy()
    assert np.all(c == 1), (np.bincount(c), np.nonzero(c != 1)[0][:10])
    st = st.cpu().numpy()
    assert np.all((st >= 0) & (st <= 3)) and np.all(it.cpu().numpy() >= 0)


@pytest.mark.parametrize("waves", [1, 2, 8])
def test_waves_per_workgroup_leave_results_bitwise_unchanged(waves):
    """A forward kernel built for another workgroup size (the waves_per_group
    option; the autotuner tries 2 and 8 waves): every cell's arithmetic is its
    slot's, so the results are bitwise those of the default four-wave
    workgroup."""
    mech, cells = config_inputs(3, ncells=20000)[0]
    V, G, B = gpu(cells["values"]), gpu(cells["gamma"]), gpu(cells["b"])
    ref = bcs.solve_batch(bcs.Plan(mech.row_ptr, mech.col_idx, lanes_per_cell=32, autotune=False), V, G, B, RTOL, 200)
    plan = bcs.Plan(mech.row_ptr, mech.col_idx, lanes_per_cell=32, autotune=False, waves_per_group=waves)
    assert plan.info()["cells_per_wg"] == 2 * waves
    got = bcs.solve_batch(plan, V, G, B, RTOL, 200)
    torch.cuda.synchronize()
    for a, b in zip(got[:4], ref[:4]):
        assert torch.equal(a, b)


@pytest.mark.parametrize("lanes", [32, 64])
def test_batch_sizes_around_the_slot_count(lanes, monkeypatch):
    """A launch gives every cell a slot of its own when the batch fits the
    resident grid (no queue), and otherwise hands out the slots' first claims
    without the counter and the rest through it.  Around each possible slot
    count (1-4 resident workgroups per CU) every cell is written exactly
    once, and every output is bitwise the same cell's output in a
    10,000-cell batch (a cell's result depends on nothing else)."""
    monkeypatch.setenv("BCS_DEBUG_VISITS", "1")
    mech, cells = config_inputs(3, ncells=10000)[0]
    V, G, B = gpu(cells["values"]), gpu(cells["gamma"]), gpu(cells["b"])
    plan = bcs.Plan(mech.row_ptr, mech.col_idx, lanes_per_cell=lanes)
    full = [t.cpu().numpy() for t in bcs.solve_batch(plan, V, G, B, RTOL, 200)[:4]]
    cpw = plan.info()["cells_per_wg"]
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    L = bcs.lib()
    sizes = sorted({c for k in (1, 2, 3, 4) for c in (cpw * ncu * k - 1, cpw * ncu * k, cpw * ncu * k + 1)
                    if c <= V.shape[0]})
    assert len(sizes) >= 6
    for C in sizes:
        counts = torch.zeros(C, dtype=torch.int32, device="cuda")
        L.bcs_debug_count_visits(counts.data_ptr())
        try:
            got = bcs.solve_batch(plan, V[:C], G[:C], B[:C], RTOL, 200)
            torch.cuda.synchronize()
        finally:
            L.bcs_debug_count_visits(None)
        c = counts.cpu().numpy()
        assert np.all(c == 1), (C, np.bincount(c))
        for a, b in zip(full, got[:4]):
            b = b.cpu().numpy()
            assert np.array_equal(a[:C], b, equal_nan=b.dtype.kind == "f"), C
