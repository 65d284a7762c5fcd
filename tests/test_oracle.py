"""Pins of the CPU oracle against facts that do not come from the oracle itself.

* dense LU against LAPACK (numpy.linalg.solve) and Cramer's rule;
* BiCGStab against dense LU on tiny random systems (kappa-scaled tolerance);
* finite termination: on a matrix whose minimal polynomial has degree k,
  BiCGStab (like the BiCG it is built on) terminates within k iterations --
  any dropped term, wrong sign or transposed operand in the recurrences
  destroys this;
* closed forms: gamma = 0 gives x = b in one half-step; a diagonal A with
  Jacobi gives x_i = b_i / A_ii in one half-step;
* the classic exact breakdown ([[0,1],[-1,0]], b = e_1);
* forced failures (NaN, maxit = 1, b = 0, singular cells);
* the mass-action conservation invariant 1^T A = 1^T on solutions;
* adjoint: LU of A^T, duality g^T x = lambda^T b, central finite differences.
"""
import numpy as np
import scipy.linalg
import pytest

import oracle
from oracle import BREAKDOWN, CONVERGED, MAXIT, NONFINITE, A_DIRECT, J_GAMMA
from workload import config_inputs, gen_cells, gen_mechanism

RNG = np.random.default_rng(20240527)


def dense_to_csr(M):
    n = M.shape[0]
    rp = [0]
    ci = []
    vals = []
    for i in range(n):
        for j in range(n):
            if M[i, j] != 0.0 or i == j:
                ci.append(j)
                vals.append(M[i, j])
        rp.append(len(ci))
    return np.array(rp, np.int32), np.array(ci, np.int32), np.array(vals)


def random_sparse(n, density, rng):
    M = np.where(rng.uniform(size=(n, n)) < density, rng.standard_normal((n, n)), 0.0)
    M[np.arange(n), np.arange(n)] = rng.uniform(1.0, 3.0, n) * rng.choice([-1, 1], n)
    return M


# ---------------------------------------------------------------- dense LU ---

def test_lu_matches_lapack():
    for n in range(1, 13):
        for _ in range(20):
            A = RNG.standard_normal((n, n))
            b = RNG.standard_normal(n)
            x, info = oracle.lu_solve_dense(A, b)
            assert info == 0
            xr = np.linalg.solve(A, b)
            assert np.linalg.norm(x - xr) <= 1e-10 * np.linalg.cond(A) * np.linalg.norm(xr)


def test_lu_matches_cramer_rule():
    def det2(M):
        return M[0, 0] * M[1, 1] - M[0, 1] * M[1, 0]

    def det3(M):
        return (M[0, 0] * (M[1, 1] * M[2, 2] - M[1, 2] * M[2, 1])
                - M[0, 1] * (M[1, 0] * M[2, 2] - M[1, 2] * M[2, 0])
                + M[0, 2] * (M[1, 0] * M[2, 1] - M[1, 1] * M[2, 0]))

    for n, det in ((2, det2), (3, det3)):
        for _ in range(50):
            A = RNG.standard_normal((n, n))
            b = RNG.standard_normal(n)
            x, _ = oracle.lu_solve_dense(A, b)
            d = det(A)
            for j in range(n):
                Aj = A.copy()
                Aj[:, j] = b
                assert abs(x[j] - det(Aj) / d) <= 1e-9 * (1 + abs(x[j])) * np.linalg.cond(A)


def test_lu_pivots_on_zero_leading_entry_and_flags_singular():
    A = np.array([[0.0, 2.0], [3.0, 1.0]])
    x, info = oracle.lu_solve_dense(A, np.array([2.0, 4.0]))
    assert info == 0 and np.allclose(x, [1.0, 1.0], rtol=0, atol=1e-15)
    _, info = oracle.lu_solve_dense(np.array([[1.0, 2.0], [2.0, 4.0]]), np.array([1.0, 1.0]))
    assert info == 2


def test_lu_batch_transpose_solves_transposed_system():
    M = random_sparse(7, 0.4, RNG)
    rp, ci, vals = dense_to_csr(M)
    b = RNG.standard_normal(7)
    x, info = oracle.lu_batch(rp, ci, vals[None], [0.0], b[None], kind=A_DIRECT, transpose=True)
    assert info[0] == 0
    assert np.allclose(x[0], np.linalg.solve(M.T, b), rtol=1e-12, atol=1e-12)


# ----------------------------------------------------- BiCGStab vs dense LU --

@pytest.mark.parametrize("precond", [0, 1])
def test_bicgstab_matches_lu_on_tiny_random_systems(precond):
    checked = 0
    for trial in range(2000):
        n = int(RNG.integers(1, 9))
        M = random_sparse(n, 0.5, RNG)
        kappa = np.linalg.cond(M)
        if kappa > 1e6:
            continue
        rp, ci, vals = dense_to_csr(M)
        b = RNG.standard_normal(n)
        x, it, res, st = oracle.solve_batch(rp, ci, vals[None], [0.0], b[None], rtol=1e-12, maxit=400,
                                            precond=precond, kind=A_DIRECT)
        xr = np.linalg.solve(M, b)
        if st[0] == BREAKDOWN:
            continue  # an exact breakdown is a legitimate outcome; covered separately
        assert st[0] == CONVERGED, (trial, it, res)
        assert res[0] <= 1e-12
        assert np.linalg.norm(x[0] - xr) <= 4 * kappa * max(res[0], 1e-15) * np.linalg.norm(xr) + 1e-14
        checked += 1
    assert checked > 1500


def test_returned_residual_is_the_true_residual():
    mech, cells = config_inputs(1)[0]
    x, it, res, st = oracle.solve_batch(mech.row_ptr, mech.col_idx, cells["values"], cells["gamma"], cells["b"],
                                        precond=1)
    for c in range(0, 100, 7):
        A = oracle.to_dense(mech.row_ptr, mech.col_idx,
                            oracle.form_a(mech.row_ptr, mech.col_idx, cells["values"][c], cells["gamma"][c]))
        r = cells["b"][c] - A @ x[c]
        rel = np.linalg.norm(r) / np.linalg.norm(cells["b"][c])
        assert abs(rel - res[c]) <= 1e-3 * rel + 1e-15


# --------------------------------------------------------- finite termination

def _eig_construct(eigs, n, rng, symmetric):
    d = np.array([eigs[i % len(eigs)] for i in range(n)])
    if symmetric:
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        return Q @ np.diag(d) @ Q.T
    Q = rng.standard_normal((n, n)) + 3 * np.eye(n)
    return Q @ np.diag(d) @ np.linalg.inv(Q)


@pytest.mark.parametrize("k,symmetric", [(1, True), (2, True), (3, True), (4, True), (5, True),
                                         (1, False), (2, False), (3, False)])
def test_finite_termination_within_degree_of_minimal_polynomial(k, symmetric):
    # For SPD A and rhat = r0, BiCG reproduces CG, so its residual polynomial
    # vanishes after k steps when A has k distinct eigenvalues; BiCGStab's
    # half-step residual s_k contains that factor and is zero too.  For
    # non-normal A the same holds in exact arithmetic; with rounding it stays
    # reliable for k <= 3 on these eigenvector matrices.
    eigs = [1.0, 2.5, 4.0, 6.0, 9.0][:k]
    for trial in range(40):
        n = 12
        M = _eig_construct(eigs, n, RNG, symmetric)
        rp, ci, vals = dense_to_csr(M)
        b = RNG.standard_normal(n)
        x, it, res, st = oracle.solve_batch(rp, ci, vals[None], [0.0], b[None], rtol=1e-9, maxit=50,
                                            kind=A_DIRECT)
        assert st[0] == CONVERGED
        assert it[0] <= k, (k, it[0])


def test_rank_one_update_converges_in_two_iterations():
    n = 40
    for _ in range(20):
        u = RNG.standard_normal(n)
        v = RNG.standard_normal(n)
        M = np.eye(n) + np.outer(u, v) / n
        if abs(1 + v @ u / n) < 0.1:
            continue
        rp, ci, vals = dense_to_csr(M)
        b = RNG.standard_normal(n)
        x, it, res, st = oracle.solve_batch(rp, ci, vals[None], [0.0], b[None], rtol=1e-10, kind=A_DIRECT)
        assert st[0] == CONVERGED and it[0] <= 2
        assert np.allclose(x[0], np.linalg.solve(M, b), rtol=1e-8, atol=1e-10)


# ------------------------------------------------------------- closed forms --

@pytest.mark.parametrize("precond", [0, 1])
def test_gamma_zero_gives_b_in_one_half_step(precond):
    mech, cells = config_inputs(1, ncells=5)[0]
    x, it, res, st = oracle.solve_batch(mech.row_ptr, mech.col_idx, cells["values"], np.zeros(5), cells["b"],
                                        precond=precond)
    assert np.all(st == CONVERGED) and np.all(it == 1)
    assert np.array_equal(x, cells["b"])
    assert np.all(res == 0.0)


def test_diagonal_with_jacobi_is_exact_in_one_step():
    n = 17
    d = RNG.uniform(1.0, 1e4, n)
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    b = RNG.standard_normal(n)
    x, it, res, st = oracle.solve_batch(rp, ci, d[None], [0.0], b[None], precond=1, kind=A_DIRECT)
    assert st[0] == CONVERGED and it[0] == 1
    assert np.allclose(x[0], b / d, rtol=4e-16, atol=0)


def test_two_species_isomerisation_closed_form():
    # A <-> B with rates k1 (A->B) and k2 (B->A): J = [[-k1, k2], [k1, -k2]].
    k1, k2, g = 3.0, 0.5, 0.7
    J = np.array([-k1, k2, k1, -k2])
    rp = np.array([0, 2, 4], np.int32)
    ci = np.array([0, 1, 0, 1], np.int32)
    b = np.array([1.0, 2.0])
    x, it, res, st = oracle.solve_batch(rp, ci, J[None], [g], b[None], rtol=1e-14)
    # (I - gJ) x = b solved by hand: det = 1 + g (k1 + k2)
    det = 1 + g * (k1 + k2)
    x0 = ((1 + g * k2) * b[0] + g * k2 * b[1]) / det
    x1 = (g * k1 * b[0] + (1 + g * k1) * b[1]) / det
    assert st[0] == CONVERGED
    assert np.allclose(x[0], [x0, x1], rtol=1e-13, atol=0)
    assert abs(x[0].sum() - b.sum()) <= 1e-13  # molecule conservation


# ------------------------------------------------- breakdown and failures ----

def test_exact_breakdown_of_rotation_matrix():
    A = np.array([0.0, 1.0, -1.0, 0.0])
    rp = np.array([0, 2, 4], np.int32)
    ci = np.array([0, 1, 0, 1], np.int32)
    b = np.array([1.0, 0.0])
    x, it, res, st = oracle.solve_batch(rp, ci, A[None], [0.0], b[None], kind=A_DIRECT)
    assert st[0] == BREAKDOWN and it[0] == 2 and np.all(x[0] == 0) and res[0] == 1.0
    # the same system in J mode: A = I - gamma J with gamma = 1, J = I - A
    J = np.array([1.0, -1.0, 1.0, 1.0])
    x2, it2, res2, st2 = oracle.solve_batch(rp, ci, J[None], [1.0], b[None])
    assert st2[0] == BREAKDOWN and it2[0] == 2
    # no restarts allowed: breakdown after one iteration
    _, it3, _, st3 = oracle.solve_batch(rp, ci, A[None], [0.0], b[None], kind=A_DIRECT, breakdown_restarts=0)
    assert st3[0] == BREAKDOWN and it3[0] == 1


def test_nan_cell_is_isolated():
    mech, cells = config_inputs(1, ncells=6)[0]
    vals = cells["values"].copy()
    vals[3, 5] = np.nan
    args = (mech.row_ptr, mech.col_idx)
    x, it, res, st = oracle.solve_batch(*args, vals, cells["gamma"], cells["b"], precond=1)
    x0, it0, res0, st0 = oracle.solve_batch(*args, cells["values"], cells["gamma"], cells["b"], precond=1)
    assert st[3] == NONFINITE
    keep = [0, 1, 2, 4, 5]
    assert np.array_equal(x[keep], x0[keep]) and np.array_equal(it[keep], it0[keep])
    b = cells["b"].copy()
    b[2, 0] = np.inf
    _, _, _, st2 = oracle.solve_batch(*args, cells["values"], cells["gamma"], b, precond=1)
    assert st2[2] == NONFINITE


def test_maxit_one_and_zero_rhs():
    mech, cells = config_inputs(1, ncells=4)[0]
    b = cells["b"].copy()
    b[1] = 0.0
    x, it, res, st = oracle.solve_batch(mech.row_ptr, mech.col_idx, cells["values"], cells["gamma"], b,
                                        maxit=1, precond=1)
    assert st[1] == CONVERGED and it[1] == 0 and res[1] == 0.0 and np.all(x[1] == 0.0)
    hard = [c for c in (0, 2, 3) if st[c] != CONVERGED]
    assert hard and all(st[c] == MAXIT and it[c] == 1 for c in hard)


def test_singular_diagonal_cell():
    n, g = 4, 0.5
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    J = np.full(n, 1.0 / g)  # A = I - g J = 0
    b = np.ones(n)
    _, _, _, st = oracle.solve_batch(rp, ci, J[None], [g], b[None], precond=0)
    assert st[0] == BREAKDOWN
    _, _, _, st = oracle.solve_batch(rp, ci, J[None], [g], b[None], precond=1)
    assert st[0] == NONFINITE


# ----------------------------------------------- mass-action workloads -------

@pytest.mark.parametrize("cfg", [1, 4])
def test_mass_action_cells_match_lu_and_conserve(cfg):
    for mech, cells in config_inputs(cfg, ncells=120):
        rp, ci = mech.row_ptr, mech.col_idx
        x, it, res, st = oracle.solve_batch(rp, ci, cells["values"], cells["gamma"], cells["b"], precond=1)
        xl, info = oracle.lu_batch(rp, ci, cells["values"], cells["gamma"], cells["b"])
        assert np.all(info == 0)
        assert np.mean(st == CONVERGED) >= 0.99
        for c in np.nonzero(st == CONVERGED)[0]:
            A = oracle.to_dense(rp, ci, oracle.form_a(rp, ci, cells["values"][c], cells["gamma"][c]))
            kappa = np.linalg.cond(A)
            rlu = np.linalg.norm(cells["b"][c] - A @ xl[c]) / np.linalg.norm(cells["b"][c])
            err = np.linalg.norm(x[c] - xl[c]) / np.linalg.norm(xl[c])
            assert err <= max(1e-8, 4 * kappa * max(res[c], rlu))
            # 1^T A = 1^T  =>  sum(x) - sum(b) = -sum(b - A x)
            bn = np.linalg.norm(cells["b"][c])
            slack = np.sqrt(mech.n) * res[c] * bn + 1e3 * np.finfo(float).eps * (np.abs(A) @ np.abs(x[c])).sum()
            assert abs(x[c].sum() - cells["b"][c].sum()) <= slack


def test_ideal_cells_give_identical_results():
    mech, cells = config_inputs(1, ncells=16, mode="ideal")[0]
    x, it, res, st = oracle.solve_batch(mech.row_ptr, mech.col_idx, cells["values"], cells["gamma"], cells["b"],
                                        precond=1)
    assert np.all(x == x[0]) and np.all(it == it[0]) and np.all(res == res[0])


def test_permuting_cells_permutes_results_bitwise():
    mech, cells = config_inputs(1, ncells=10)[0]
    perm = RNG.permutation(10)
    a = oracle.solve_batch(mech.row_ptr, mech.col_idx, cells["values"], cells["gamma"], cells["b"], precond=1)
    b = oracle.solve_batch(mech.row_ptr, mech.col_idx, cells["values"][perm], cells["gamma"][perm],
                           cells["b"][perm], precond=1)
    for u, v in zip(a, b):
        assert np.array_equal(u[perm], v)


# ------------------------------------------------------- Block-cells (N) ----

def test_block_pattern_is_the_block_diagonal_matrix():
    mech, cells = config_inputs(1, ncells=3)[0]
    rp, ci = mech.row_ptr, mech.col_idx
    rpg, cig = oracle.block_pattern(rp, ci, 3)
    dense = oracle.to_dense(rpg, cig, cells["values"].reshape(-1))
    want = scipy.linalg.block_diag(*[oracle.to_dense(rp, ci, v) for v in cells["values"]])
    assert np.array_equal(dense, want)


def test_groups_of_one_are_the_per_cell_solves():
    mech, cells = config_inputs(1, ncells=30)[0]
    args = (mech.row_ptr, mech.col_idx, cells["values"], cells["gamma"], cells["b"])
    x, it, res, st = oracle.solve_batch(*args, precond=1)
    xg, itg, resg, stg = oracle.solve_groups(*args, group=1, precond=1)
    assert np.array_equal(x, xg) and np.array_equal(it, itg) and np.array_equal(st, stg)
    # the same residual, summed in another order: equal within its rounding
    for c in range(30):
        A = oracle.to_dense(mech.row_ptr, mech.col_idx,
                            oracle.form_a(mech.row_ptr, mech.col_idx, cells["values"][c], cells["gamma"][c]))
        slack = 64 * np.finfo(float).eps * np.linalg.norm(np.abs(A) @ np.abs(x[c])) / np.linalg.norm(cells["b"][c])
        assert abs(res[c] - resg[c]) <= slack


@pytest.mark.parametrize("group", [2, 4])
def test_identical_cells_in_a_run_iterate_like_one_cell(group):
    """A run of identical cells has every inner product `group` times the one
    cell's (up to rounding), so alpha, omega, beta and the iterates are the
    one cell's: same iteration count (within one) and the same x."""
    mech, cells = config_inputs(1, ncells=8, mode="ideal")[0]
    args = (mech.row_ptr, mech.col_idx, cells["values"], cells["gamma"], cells["b"])
    x, it, res, st = oracle.solve_batch(*args, precond=1)
    xg, itg, resg, stg = oracle.solve_groups(*args, group=group, precond=1)
    assert np.all(np.abs(itg - it) <= 1)
    assert np.all(np.linalg.norm(xg - x, axis=1) <= 1e-8 * np.linalg.norm(x, axis=1))


def test_runs_are_independent_and_the_last_run_may_be_short():
    """Cells 0..5 in runs of 4 are runs {0..3} and {4, 5}: solving {4, 5} alone
    as one run of 2 gives the same results bitwise."""
    mech, cells = config_inputs(1, ncells=6)[0]
    rp, ci = mech.row_ptr, mech.col_idx
    full = oracle.solve_groups(rp, ci, cells["values"], cells["gamma"], cells["b"], group=4, precond=1)
    tail = oracle.solve_groups(rp, ci, cells["values"][4:], cells["gamma"][4:], cells["b"][4:], group=2, precond=1)
    for u, v in zip(full, tail):
        assert np.array_equal(u[4:], v)


def test_grouped_cells_meet_the_lu_bound():
    mech, cells = config_inputs(1, ncells=40)[0]
    rp, ci = mech.row_ptr, mech.col_idx
    x, it, res, st = oracle.solve_groups(rp, ci, cells["values"], cells["gamma"], cells["b"], group=4, precond=1)
    xl, _ = oracle.lu_batch(rp, ci, cells["values"], cells["gamma"], cells["b"])
    assert np.mean(st == 0) >= 0.9
    for c in np.nonzero(st == 0)[0]:
        A = oracle.to_dense(rp, ci, oracle.form_a(rp, ci, cells["values"][c], cells["gamma"][c]))
        kappa = np.linalg.cond(A)
        rlu = np.linalg.norm(cells["b"][c] - A @ xl[c]) / np.linalg.norm(cells["b"][c])
        assert res[c] <= 1e-10
        assert np.linalg.norm(x[c] - xl[c]) / np.linalg.norm(xl[c]) <= max(1e-8, 4 * kappa * max(res[c], rlu))
    # the cells of a run report the run's iteration count
    assert np.all(it.reshape(10, 4) == it.reshape(10, 4)[:, :1])


# ------------------------------------------------------------------ adjoint --

def _loss_lu(rp, ci, vals, gamma, b, w):
    x, info = oracle.lu_batch(rp, ci, vals[None], [gamma], b[None])
    return float(w @ x[0])


def test_adjoint_matches_transposed_lu_and_duality():
    mech, cells = config_inputs(5, ncells=40)[0]
    rp, ci = mech.row_ptr, mech.col_idx
    x, _, _, st = oracle.solve_batch(rp, ci, cells["values"], cells["gamma"], cells["b"], precond=1)
    w = cells["w"]
    gb, gA, it, res, sta = oracle.adjoint_batch(rp, ci, cells["values"], cells["gamma"], x, w, precond=1)
    lam_lu, info = oracle.lu_batch(rp, ci, cells["values"], cells["gamma"], w, transpose=True)
    for c in range(40):
        if sta[c] != CONVERGED or st[c] != CONVERGED:
            continue
        A = oracle.to_dense(rp, ci, oracle.form_a(rp, ci, cells["values"][c], cells["gamma"][c]))
        kappa = np.linalg.cond(A)
        err = np.linalg.norm(gb[c] - lam_lu[c]) / np.linalg.norm(lam_lu[c])
        assert err <= max(1e-8, 4 * kappa * res[c] + 1e-12 * kappa)
        # duality: w^T x = lambda^T b (both equal w^T A^-1 b)
        lhs, rhs = w[c] @ x[c], gb[c] @ cells["b"][c]
        scale = np.linalg.norm(w[c]) * np.linalg.norm(x[c]) + np.linalg.norm(gb[c]) * np.linalg.norm(cells["b"][c])
        assert abs(lhs - rhs) <= 1e-8 * scale
        # pattern gradient is -lambda_i x_j
        for i in range(0, mech.n, 13):
            for k in range(rp[i], rp[i + 1]):
                assert gA[c, k] == -gb[c, i] * x[c, ci[k]]


def test_adjoint_matches_central_finite_differences():
    mech, cells = config_inputs(5, ncells=12)[0]
    rp, ci = mech.row_ptr, mech.col_idx
    rng = np.random.Generator(np.random.PCG64(5))
    for c in rng.choice(12, size=4, replace=False):
        vals, g, b, w = cells["values"][c], cells["gamma"][c], cells["b"][c], cells["w"][c]
        A = oracle.form_a(rp, ci, vals, g)
        x, _ = oracle.lu_batch(rp, ci, A[None], [0.0], b[None], kind=A_DIRECT)
        gb, gA, it, res, st = oracle.adjoint_batch(rp, ci, A[None], [0.0], x, w[None], rtol=1e-12, precond=1,
                                                   kind=A_DIRECT)
        amax = np.abs(gA[0]).max()

        def L(Av, bv):
            xx, _ = oracle.lu_batch(rp, ci, Av[None], [0.0], bv[None], kind=A_DIRECT)
            return float(w @ xx[0])

        L0 = abs(L(A, b))
        # a relative step 1e-6*|A_k| moves L by about 1e-6*|A_k*dL/dA_k|; keep
        # entries where that is far above the rounding of L (about 1e-16*|L|)
        resolvable = np.nonzero(1e-6 * np.abs(A * gA[0]) > 1e-8 * L0)[0]
        assert resolvable.size >= 12
        for k in rng.choice(resolvable, size=12, replace=False):
            eps = 1e-6 * abs(A[k])
            Ap, Am = A.copy(), A.copy()
            Ap[k] += eps
            Am[k] -= eps
            fd = (L(Ap, b) - L(Am, b)) / (2 * eps)
            assert abs(fd - gA[0, k]) <= 1e-5 * max(abs(gA[0, k]), 1e-3 * amax), (k, fd, gA[0, k])
        for i in rng.choice(mech.n, size=6, replace=False):
            e = np.zeros(mech.n)
            e[i] = 1e-6
            fd = (L(A, b + e) - L(A, b - e)) / 2e-6
            assert abs(fd - gb[0, i]) <= 1e-5 * max(abs(gb[0, i]), 1e-3 * np.abs(gb[0]).max())


# -------------------------------------------------------------- mixed form ---

def test_mixed_reaches_fp64_residual_on_well_conditioned_cells():
    mech, cells = config_inputs(1)[0]
    rp, ci = mech.row_ptr, mech.col_idx
    xm, itm, ref, res, st = oracle.mixed_batch(rp, ci, cells["values"], cells["gamma"], cells["b"])
    xl, _ = oracle.lu_batch(rp, ci, cells["values"], cells["gamma"], cells["b"])
    ok = st == CONVERGED
    assert ok.mean() >= 0.9
    assert np.all(res[ok] <= 1e-10)
    assert np.all(ref[ok] >= 2)  # FP32 alone cannot reach 1e-10
    for c in np.nonzero(ok)[0]:
        A = oracle.to_dense(rp, ci, oracle.form_a(rp, ci, cells["values"][c], cells["gamma"][c]))
        kappa = np.linalg.cond(A)
        err = np.linalg.norm(xm[c] - xl[c]) / np.linalg.norm(xl[c])
        assert err <= max(1e-8, 4 * kappa * 1e-10)


def test_mixed_refinement_count_on_rank_one_update():
    # eigenvalues {1, 1 + v.u/n}: each FP32 inner solve is exact to FP32
    # rounding, so every refinement gains about 7 digits: 1e-10 needs <= 3.
    n = 30
    u = RNG.standard_normal(n)
    v = np.abs(RNG.standard_normal(n))
    M = np.eye(n) + np.outer(np.abs(u), v) / n
    rp, ci, vals = dense_to_csr(M)
    b = RNG.standard_normal(n)
    x, it, ref, res, st = oracle.mixed_batch(rp, ci, vals[None], [0.0], b[None], kind=A_DIRECT)
    assert st[0] == CONVERGED and 2 <= ref[0] <= 3 and res[0] <= 1e-10
    assert np.allclose(x[0], np.linalg.solve(M, b), rtol=1e-9, atol=1e-12)


def test_mixed_zero_rhs_and_nan():
    mech, cells = config_inputs(1, ncells=3)[0]
    b = cells["b"].copy()
    b[0] = 0
    vals = cells["values"].copy()
    vals[2, 0] = np.nan
    x, it, ref, res, st = oracle.mixed_batch(mech.row_ptr, mech.col_idx, vals, cells["gamma"], b)
    assert st[0] == CONVERGED and ref[0] == 0 and np.all(x[0] == 0)
    assert st[2] == NONFINITE


# ----------------------------------------------------------- initial guess --

def test_initial_guess_at_the_solution_takes_no_iteration():
    mech, cells = config_inputs(1, ncells=20)[0]
    rp, ci = mech.row_ptr, mech.col_idx
    xl, _ = oracle.lu_batch(rp, ci, cells["values"], cells["gamma"], cells["b"])
    x, it, res, st = oracle.solve_batch(rp, ci, cells["values"], cells["gamma"], cells["b"], precond=1, x0=xl)
    for c in range(20):
        A = oracle.to_dense(rp, ci, oracle.form_a(rp, ci, cells["values"][c], cells["gamma"][c]))
        rlu = np.linalg.norm(cells["b"][c] - A @ xl[c]) / np.linalg.norm(cells["b"][c])
        if rlu <= 1e-10:  # the LU solution meets rtol: returned as is, no iteration
            assert st[c] == CONVERGED and it[c] == 0 and np.array_equal(x[c], xl[c])
            # the same residual, summed in another order
            slack = 64 * np.finfo(float).eps * np.linalg.norm(np.abs(A) @ np.abs(xl[c])) / np.linalg.norm(cells["b"][c])
            assert abs(res[c] - rlu) <= slack


def test_initial_guess_solves_for_the_correction():
    """BiCGStab from x0 on A x = b is BiCGStab from 0 on A e = b - A x0 with
    x = x0 + e (the Krylov space of r0): the same iteration count (rounding
    may move it by one) and x within the residual-implied bound of the LU
    solution."""
    mech, cells = config_inputs(1, ncells=40)[0]
    rp, ci = mech.row_ptr, mech.col_idx
    rng = np.random.default_rng(4)
    xl, _ = oracle.lu_batch(rp, ci, cells["values"], cells["gamma"], cells["b"])
    x0 = xl * (1 + 1e-3 * rng.standard_normal(xl.shape))
    x, it, res, st = oracle.solve_batch(rp, ci, cells["values"], cells["gamma"], cells["b"], precond=1, x0=x0)
    agree = 0
    for c in range(40):
        A = oracle.to_dense(rp, ci, oracle.form_a(rp, ci, cells["values"][c], cells["gamma"][c]))
        r0 = cells["b"][c] - A @ x0[c]
        scale = np.linalg.norm(cells["b"][c]) / np.linalg.norm(r0)
        e, ite, rese, ste = oracle.solve_batch(rp, ci, cells["values"][c][None], [cells["gamma"][c]], r0[None],
                                               rtol=1e-10 * scale, precond=1)
        agree += abs(int(ite[0]) - int(it[c])) <= 1
        if st[c] == CONVERGED:
            kappa = np.linalg.cond(A)
            err = np.linalg.norm(x[c] - xl[c]) / np.linalg.norm(xl[c])
            assert err <= max(1e-8, 4 * kappa * res[c]), (c, err)
            assert res[c] <= 1e-10
    assert agree >= 38
    # a warm start needs fewer iterations than a cold one on these cells
    _, it_cold, _, _ = oracle.solve_batch(rp, ci, cells["values"], cells["gamma"], cells["b"], precond=1)
    assert it.mean() < it_cold.mean()


def test_zero_initial_guess_equals_no_initial_guess():
    mech, cells = config_inputs(1, ncells=15)[0]
    args = (mech.row_ptr, mech.col_idx, cells["values"], cells["gamma"], cells["b"])
    a = oracle.solve_batch(*args, precond=1)
    # x0 = 0 forms r0 = b - A 0 = b exactly
    b = oracle.solve_batch(*args, precond=1, x0=np.zeros_like(cells["b"]))
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_mixed_initial_guess_at_the_solution_takes_no_refinement():
    mech, cells = config_inputs(1, ncells=10)[0]
    rp, ci = mech.row_ptr, mech.col_idx
    xl, _ = oracle.lu_batch(rp, ci, cells["values"], cells["gamma"], cells["b"])
    x, it, ref, res, st = oracle.mixed_batch(rp, ci, cells["values"], cells["gamma"], cells["b"], x0=xl)
    done = res <= 1e-10
    assert done.sum() >= 8
    assert np.all(st[done] == CONVERGED) and np.all(it[done] == 0) and np.all(ref[done] == 0)
    assert np.array_equal(x[done], xl[done])


# ------------------------------------------ the FP32 inner solver on its own --

@pytest.mark.parametrize("k", [1, 2, 3])
def test_fp32_solver_finite_termination(k):
    """In FP32 too, an SPD matrix with k distinct eigenvalues gives termination
    within k iterations (the residual polynomial of degree k vanishes on the
    spectrum); a dropped term or wrong sign in the FP32 recurrences breaks it."""
    eigs = [1.0, 2.5, 4.0][:k]
    rng = np.random.default_rng(100 + k)
    n = 12
    for trial in range(20):
        M = _eig_construct(eigs, n, rng, True)
        rp, ci, vals = dense_to_csr(M)
        b = rng.standard_normal(n)
        x, it, res, st = oracle.solve_batch_f(rp, ci, vals[None].astype(np.float32), b[None].astype(np.float32),
                                              rtol=1e-5, maxit=50)
        assert st[0] == CONVERGED and it[0] <= k, (k, it[0], res[0])
        xr = np.linalg.solve(M, b)
        assert np.linalg.norm(x[0] - xr) <= 1e-4 * np.linalg.norm(xr)


def test_fp32_solver_identity_gives_b_exactly_in_one_half_step():
    """A = I: alpha = (b, b) / (b, I b) is exactly 1 in any precision, s = 0,
    so x = b in one half step."""
    n = 30
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    b = np.random.default_rng(8).standard_normal((5, n)).astype(np.float32)
    x, it, res, st = oracle.solve_batch_f(rp, ci, np.ones((5, n), np.float32), b, rtol=1e-6)
    assert np.all(st == CONVERGED) and np.all(it == 1) and np.array_equal(x, b)


def test_fp32_solver_meets_the_fp32_bound_on_tiny_systems():
    rng = np.random.default_rng(21)
    checked = 0
    for trial in range(400):
        n = int(rng.integers(1, 9))
        M = random_sparse(n, 0.5, rng)
        kappa = np.linalg.cond(M)
        if kappa > 1e3:
            continue
        rp, ci, vals = dense_to_csr(M)
        M32 = oracle.to_dense(rp, ci, vals.astype(np.float32).astype(np.float64))
        b = rng.standard_normal(n).astype(np.float32)
        x, it, res, st = oracle.solve_batch_f(rp, ci, vals[None].astype(np.float32), b[None], rtol=1e-5, maxit=100)
        if st[0] == BREAKDOWN:
            continue
        assert st[0] == CONVERGED and res[0] <= 1e-5
        xr = np.linalg.solve(M32, b.astype(np.float64))
        # residual-implied bound plus the FP32 evaluation of the residual
        assert np.linalg.norm(x[0] - xr) <= 4 * kappa * (1e-5 + 64 * 2.0 ** -24) * np.linalg.norm(xr)
        checked += 1
    assert checked > 250


def test_mixed_budget_per_cell_never_spends_more_than_maxit():
    mech, cells = config_inputs(3, ncells=300)[0]
    rp, ci = mech.row_ptr, mech.col_idx
    args = (rp, ci, cells["values"], cells["gamma"], cells["b"])
    _, it_c, ref_c, res_c, st_c = oracle.mixed_batch(*args, maxit=200, budget="cell")
    _, it_i, ref_i, res_i, st_i = oracle.mixed_batch(*args, maxit=200, budget="inner")
    assert it_c.max() <= 200 and it_i.max() <= 200 * 10
    assert np.all(ref_i <= 10) and np.all(ref_c <= 10)
    # the per-inner-solve budget never solves fewer cells: every cell the
    # per-cell budget solves within 200 iterations, it solves the same way
    assert np.all(st_i[st_c == CONVERGED] == CONVERGED)
    assert (st_i == CONVERGED).sum() >= (st_c == CONVERGED).sum()


# ------------------------------------------------------------------ ILU(0) --

def _ilu_dense(rp, ci, F):
    n = len(rp) - 1
    M = oracle.to_dense(rp, ci, F)
    L = np.tril(M, -1) + np.eye(n)
    U = np.triu(M)
    return L, U


@pytest.mark.parametrize("source", ["random", "mechanism"])
def test_ilu0_product_equals_a_on_the_pattern(source):
    """The defining property of ILU(0): (L U)_ij = a_ij wherever (i, j) is in
    the pattern (L unit lower, U upper, both on A's pattern)."""
    rng = np.random.default_rng(31)
    cases = []
    if source == "random":
        for _ in range(60):
            n = int(rng.integers(2, 14))
            M = random_sparse(n, 0.35, rng)
            M[np.arange(n), np.arange(n)] = np.abs(M).sum(1) + rng.uniform(0.5, 2, n)
            cases.append(dense_to_csr(M))
    else:
        mech, cells = config_inputs(3, ncells=30)[0]
        for c in range(30):
            cases.append((mech.row_ptr, mech.col_idx,
                          oracle.form_a(mech.row_ptr, mech.col_idx, cells["values"][c], cells["gamma"][c])))
    for rp, ci, vals in cases:
        F = oracle.ilu0(rp, ci, vals)
        L, U = _ilu_dense(rp, ci, F)
        LU = L @ U
        rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
        got = LU[rows, ci]
        scale = (np.abs(L) @ np.abs(U))[rows, ci]
        assert np.all(np.abs(got - vals) <= 64 * np.finfo(float).eps * scale)


def test_ilu0_of_a_dense_pattern_is_lu_without_pivoting():
    """On a full pattern ILU(0) drops nothing: it is Gaussian elimination
    without pivoting, which for a diagonally dominant matrix is what LAPACK's
    partially pivoted LU computes (its permutation is the identity)."""
    rng = np.random.default_rng(32)
    for n in (3, 6, 11):
        M = rng.standard_normal((n, n))
        M[np.arange(n), np.arange(n)] = np.abs(M).sum(1) + 1.0
        rp, ci, vals = dense_to_csr(M)
        F = oracle.ilu0(rp, ci, vals)
        L, U = _ilu_dense(rp, ci, F)
        Pm, Ls, Us = scipy.linalg.lu(M)
        assert np.array_equal(Pm, np.eye(n))
        assert np.allclose(L, Ls, rtol=1e-12, atol=1e-14) and np.allclose(U, Us, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("shape", ["tridiagonal", "lower", "upper_bidiagonal"])
def test_ilu0_without_fill_is_exact_and_solves_in_one_iteration(shape):
    """Patterns on which elimination creates no fill: ILU(0) is the exact LU,
    so the exactly applied preconditioner is A^-1 and preconditioned BiCGStab
    stops at the first half step with x = A^-1 b."""
    rng = np.random.default_rng(33)
    n = 15
    M = np.diag(rng.uniform(2, 4, n))
    if shape == "tridiagonal":
        M += np.diag(rng.uniform(-1, 1, n - 1), 1) + np.diag(rng.uniform(-1, 1, n - 1), -1)
    elif shape == "lower":
        M += np.tril(rng.uniform(-1, 1, (n, n)), -1)
    else:
        M += np.diag(rng.uniform(-1, 1, n - 1), 1)
    rp, ci, vals = dense_to_csr(M)
    F = oracle.ilu0(rp, ci, vals)
    L, U = _ilu_dense(rp, ci, F)
    assert np.allclose(L @ U, M, rtol=1e-13, atol=1e-14)
    b = rng.standard_normal(n)
    x, it, res, st = oracle.solve_batch(rp, ci, vals[None], [0.0], b[None], precond=2, ilu_sweeps=0,
                                        kind=A_DIRECT)
    assert st[0] == CONVERGED and it[0] == 1
    assert np.allclose(x[0], np.linalg.solve(M, b), rtol=1e-12, atol=1e-14)


def test_ilu_sweeps_are_the_truncated_neumann_series_and_exact_at_depth():
    """s Jacobi sweeps on the unit lower triangle give y = sum_{t<=s} (-L)^t p,
    on the upper triangle z = sum_{t<=s} (-D^-1 U)^t D^-1 y; at s >= depth - 1
    both are the exact substitutions (strictly triangular parts are
    nilpotent)."""
    mech, cells = config_inputs(1, ncells=3)[0]
    rp, ci = mech.row_ptr, mech.col_idx
    n = mech.n
    A = oracle.form_a(rp, ci, cells["values"][1], cells["gamma"][1])
    F = oracle.ilu0(rp, ci, A)
    L, U = _ilu_dense(rp, ci, F)
    Ls = L - np.eye(n)
    d = np.diag(U)
    Us = np.triu(U, 1)
    p = np.random.default_rng(34).standard_normal(n)
    for s in (1, 2, 3):
        y = sum(np.linalg.matrix_power(-Ls, t) @ p for t in range(s + 1))
        K = -Us / d[:, None]
        z = sum(np.linalg.matrix_power(K, t) @ (y / d) for t in range(s + 1))
        got = oracle.ilu_apply(rp, ci, F, p, sweeps=s)
        assert np.allclose(got, z, rtol=1e-10, atol=1e-12 * np.abs(z).max())
    exact = scipy.linalg.solve_triangular(U, scipy.linalg.solve_triangular(L, p, lower=True, unit_diagonal=True))
    assert np.allclose(oracle.ilu_apply(rp, ci, F, p, sweeps=0), exact, rtol=1e-10, atol=1e-12 * np.abs(exact).max())
    assert np.allclose(oracle.ilu_apply(rp, ci, F, p, sweeps=n), exact, rtol=1e-10, atol=1e-12 * np.abs(exact).max())


def test_ilu_preconditioned_solves_match_lu_with_far_fewer_iterations():
    mech, cells = config_inputs(3, ncells=300)[0]
    rp, ci = mech.row_ptr, mech.col_idx
    args = (rp, ci, cells["values"], cells["gamma"], cells["b"])
    x, it, res, st = oracle.solve_batch(*args, precond=2, ilu_sweeps=3)
    _, itj, _, stj = oracle.solve_batch(*args, precond=1)
    xl, _ = oracle.lu_batch(*args)
    assert np.mean(st == CONVERGED) >= np.mean(stj == CONVERGED)
    both = (st == 0) & (stj == 0)
    assert it[both].mean() < 0.4 * itj[both].mean()
    for c in np.nonzero(st == CONVERGED)[0][::5]:
        A = oracle.to_dense(rp, ci, oracle.form_a(rp, ci, cells["values"][c], cells["gamma"][c]))
        kappa = np.linalg.cond(A)
        rlu = np.linalg.norm(cells["b"][c] - A @ xl[c]) / np.linalg.norm(cells["b"][c])
        err = np.linalg.norm(x[c] - xl[c]) / np.linalg.norm(xl[c])
        assert err <= max(1e-8, 4 * kappa * max(res[c], rlu))


# ------------------------------------------- mass-action rates and Jacobian ----
# The oracle's assembly (oracle_assemble) is pinned by a hand-computed
# example, by the generator's independent Python implementation
# (workload.rates / workload.jacobian_values), by the mechanism's structural
# invariants (molecule count conserved: zero column sums of J and zero sum of
# f; no autocatalysis: J_ii <= 0) and by central differences of f, which are
# exact up to rounding because f is at most quadratic in y.

def test_assemble_hand_example():
    # species 0, 1, 2: 0 -> 1 (k = 2); 0 + 1 -> 2 + 2 (k = 3); 2 + 2 -> 0 + 1 (k = 5)
    reac = [[0, -1], [0, 1], [2, 2]]
    prod = [[1, -1], [2, 2], [0, 1]]
    rp = np.array([0, 3, 6, 9], np.int32)
    ci = np.array([0, 1, 2] * 3, np.int32)
    y = np.array([[1.0, 2.0, 3.0]])
    f, J = oracle.assemble(reac, prod, [2.0, 3.0, 5.0], rp, ci, y)
    # w = 2 * 1, 3 * 1 * 2, 5 * 3 * 3 = 2, 6, 45
    assert f.tolist() == [[-2 - 6 + 45, 2 - 6 + 45, 2 * 6 - 2 * 45]]
    # dw0/dy0 = 2; dw1/dy0 = 3 y1 = 6, dw1/dy1 = 3 y0 = 3; dw2/dy2 = 2 * 5 * y2 = 30
    assert J.reshape(3, 3).tolist() == [[-8, -3, 30], [-4, -3, 30], [12, 6, -60]]


@pytest.mark.parametrize("n,R", [(30, 50), (80, 150), (200, 400)])
def test_assemble_matches_the_generator(n, R):
    m = gen_mechanism(n, R)
    y = gen_cells(m, 40, 11)["y"]
    f, J = oracle.assemble(m.reactants, m.products, m.k, m.row_ptr, m.col_idx, y)
    from workload import jacobian_values, rates
    assert np.array_equal(J, jacobian_values(m, y))
    fr = rates(m, y)
    assert np.all(np.abs(f - fr) <= 1e-14 * np.abs(fr) + 1e-300)


@pytest.mark.parametrize("n,R", [(30, 50), (80, 150)])
def test_assemble_invariants(n, R):
    m = gen_mechanism(n, R)
    y = gen_cells(m, 40, 12)["y"]
    f, J = oracle.assemble(m.reactants, m.products, m.k, m.row_ptr, m.col_idx, y)
    rows = np.repeat(np.arange(n), np.diff(m.row_ptr))
    colsum = np.zeros((40, n))
    colabs = np.zeros((40, n))
    np.add.at(colsum.T, m.col_idx, J.T)
    np.add.at(colabs.T, m.col_idx, np.abs(J).T)
    u = np.finfo(np.float64).eps / 2
    assert np.all(np.abs(colsum) <= 64 * u * colabs)
    assert np.all(np.abs(f.sum(1)) <= 1e-12 * np.abs(f).sum(1))
    assert np.all(J[:, rows == m.col_idx] <= 0)


def test_assemble_central_differences_are_exact_up_to_rounding():
    m = gen_mechanism(30, 50)
    y = gen_cells(m, 3, 13)["y"]
    f, J = oracle.assemble(m.reactants, m.products, m.k, m.row_ptr, m.col_idx, y)
    Jd = np.stack([oracle.to_dense(m.row_ptr, m.col_idx, J[c]) for c in range(3)])
    for j in range(m.n):
        h = 1e-3 * y[:, j]
        yp, ym = y.copy(), y.copy()
        yp[:, j] += h
        ym[:, j] -= h
        fp, _ = oracle.assemble(m.reactants, m.products, m.k, m.row_ptr, m.col_idx, yp)
        fm, _ = oracle.assemble(m.reactants, m.products, m.k, m.row_ptr, m.col_idx, ym)
        cd = (fp - fm) / (2 * h[:, None])
        scale = (np.abs(fp) + np.abs(fm) + np.abs(f)).max(1, keepdims=True) / h[:, None]
        assert np.all(np.abs(cd - Jd[:, :, j]) <= 1e-12 * scale + 1e-9 * np.abs(Jd[:, :, j]))


def test_assemble_per_cell_rate_constants():
    m = gen_mechanism(30, 50)
    y = gen_cells(m, 4, 14)["y"]
    f1, J1 = oracle.assemble(m.reactants, m.products, m.k, m.row_ptr, m.col_idx, y)
    kc = np.stack([m.k * 2.0 ** c for c in range(4)])  # power-of-two scaling is exact
    f2, J2 = oracle.assemble(m.reactants, m.products, kc, m.row_ptr, m.col_idx, y)
    for c in range(4):
        assert np.array_equal(f2[c], f1[c] * 2.0 ** c) and np.array_equal(J2[c], J1[c] * 2.0 ** c)


def test_assemble_rejects_a_pattern_without_the_entries():
    m = gen_mechanism(30, 50)
    rp = np.arange(31, dtype=np.int32)  # diagonal only
    ci = np.arange(30, dtype=np.int32)
    with pytest.raises(ValueError):
        oracle.assemble(m.reactants, m.products, m.k, rp, ci, np.ones((1, 30)))
