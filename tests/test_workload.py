"""Pins of the synthetic mass-action generator (inputs shared by oracle and GPU).

Checks against chemistry/mathematics facts rather than against the code:
molecule-count conservation gives zero column sums of J, no autocatalysis
gives J_ii <= 0, and a quadratic f makes a central difference exact.
"""
import numpy as np
import pytest

from workload import config_inputs, gen_cells, gen_mechanism, jacobian_values, rates


@pytest.mark.parametrize("n,R", [(30, 50), (80, 150), (200, 400)])
def test_pattern_is_valid_csr_with_diagonal(n, R):
    m = gen_mechanism(n, R)
    assert m.row_ptr[0] == 0 and m.row_ptr[-1] == m.nnz
    for i in range(n):
        cols = m.col_idx[m.row_ptr[i]:m.row_ptr[i + 1]]
        assert np.all(np.diff(cols) > 0)
        assert i in cols
        assert cols.min() >= 0 and cols.max() < n


def test_n80_density_in_range():
    m = gen_mechanism(80, 150)
    assert 8.0 <= m.nnz / 80 <= 12.0


def test_reactions_conserve_molecules_and_are_not_autocatalytic():
    m = gen_mechanism(80, 150)
    for r in range(m.R):
        reac = [s for s in m.reactants[r] if s >= 0]
        prod = [s for s in m.products[r] if s >= 0]
        assert len(reac) == len(prod)
        assert not set(reac) & set(prod)


def test_jacobian_column_sums_vanish():
    m = gen_mechanism(80, 150)
    cells = gen_cells(m, 50, seed=7)
    J = cells["values"]
    dense_cols = np.zeros((50, m.n))
    abs_cols = np.zeros((50, m.n))
    for i in range(m.n):
        for k in range(m.row_ptr[i], m.row_ptr[i + 1]):
            dense_cols[:, m.col_idx[k]] += J[:, k]
            abs_cols[:, m.col_idx[k]] += np.abs(J[:, k])
    assert np.all(np.abs(dense_cols) <= 64 * np.finfo(float).eps * abs_cols + 1e-300)


def test_jacobian_diagonal_nonpositive():
    m = gen_mechanism(80, 150)
    J = gen_cells(m, 20, seed=3)["values"]
    assert np.all(J[:, m.diag_pos()] <= 0.0)


def test_jacobian_matches_central_difference_exactly():
    # f is at most quadratic in y, so (f(y+h e_j) - f(y-h e_j)) / 2h has no
    # truncation error: only rounding separates it from column j of J.
    m = gen_mechanism(30, 50)
    rng = np.random.default_rng(0)
    y = 10.0 ** rng.uniform(-1, 1, size=m.n)
    J = jacobian_values(m, y[None, :])[0]
    Jd = np.zeros((m.n, m.n))
    for i in range(m.n):
        Jd[i, m.col_idx[m.row_ptr[i]:m.row_ptr[i + 1]]] = J[m.row_ptr[i]:m.row_ptr[i + 1]]
    h = 0.25  # exactly representable, so y +- h e_j is formed with one rounding
    fscale = np.abs(rates(m, y)).max() + np.abs(J).max() * np.abs(y).max()
    for j in range(m.n):
        e = np.zeros(m.n)
        e[j] = h
        fd = (rates(m, y + e) - rates(m, y - e)) / (2 * h)
        assert np.allclose(fd, Jd[:, j], rtol=0, atol=1e-12 * fscale / h)
    # entries outside the pattern are structurally zero
    off = ~m.dense_pattern()
    assert np.all(Jd[off] == 0.0)


def test_ideal_mode_gives_identical_cells():
    m = gen_mechanism(30, 50)
    c = gen_cells(m, 9, seed=11, mode="ideal")
    for key in ("values", "gamma", "b"):
        assert np.all(c[key] == c[key][0])


def test_seeded_draws_are_reproducible():
    a = config_inputs(1)[0][1]
    b = config_inputs(1)[0][1]
    for key in ("values", "gamma", "b"):
        assert np.array_equal(a[key], b[key])
    g = a["gamma"]
    assert g.min() >= 0.5e-3 and g.max() <= 0.5 * 10.0


def test_config4_cell_split_is_one_two_one():
    cfg = config_inputs(4, ncells=400)
    assert [m.n for m, _ in cfg] == [30, 80, 200]
    assert [c["b"].shape[0] for _, c in cfg] == [100, 200, 100]
