"""GPU parity of the on-device mass-action assembly (rates f and Jacobian J)
against the CPU oracle's assembly.

Every sum of the assembly is taken over reactions in increasing order with one
rounding per term (the stoichiometric factor times the rounded rate or
derivative is exact), on both sides, so the bar is bitwise equality: the
benchmark workload's 100,000 cells, all three mechanisms of the uneven batch
(n = 30, 80, 200), per-cell rate constants, non-finite concentrations, and
the empty batch.  The Jacobian assembled on the device also reproduces the
workload generator's values bitwise and, fed to the solver, its solutions."""
import numpy as np
import pytest

import oracle
from workload import config_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - collected on CPU hosts too
    pytest.skip("no GPU", allow_module_level=True)

import paper_2405_17363_amd as bcs  # noqa: E402


def gpu(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def mech_of(m):
    return bcs.Mechanism(m.n, m.reactants, m.products, m.row_ptr, m.col_idx)


def same(a, b):
    return np.array_equal(a, b, equal_nan=True) and np.array_equal(np.signbit(a), np.signbit(b))


def test_config3_full_size_bitwise():
    m, cells = config_inputs(3)[0]
    M = mech_of(m)
    f, J = bcs.assemble(M, gpu(cells["y"]), gpu(m.k))
    torch.cuda.synchronize()
    f, J = f.cpu().numpy(), J.cpu().numpy()
    fo, Jo = oracle.assemble(m.reactants, m.products, m.k, m.row_ptr, m.col_idx, cells["y"])
    assert same(J, Jo) and same(f, fo)
    assert np.array_equal(J, cells["values"])  # the generator's own values


def test_config4_mechanisms_and_per_cell_rate_constants():
    for m, cells in config_inputs(4, ncells=6000):
        M = mech_of(m)
        C = cells["y"].shape[0]
        kc = m.k[None, :] * 10.0 ** np.random.default_rng(m.n).uniform(-1, 1, size=(C, m.R))
        for k in (m.k, kc):
            f, J = bcs.assemble(M, gpu(cells["y"]), gpu(k))
            torch.cuda.synchronize()
            fo, Jo = oracle.assemble(m.reactants, m.products, k, m.row_ptr, m.col_idx, cells["y"])
            assert same(J.cpu().numpy(), Jo), m.n
            assert same(f.cpu().numpy(), fo), m.n


def test_outputs_selected_edge_values_and_empty_batch():
    m, cells = config_inputs(1)[0]
    M = mech_of(m)
    y = cells["y"].copy()
    y[3, 5] = np.nan
    y[4, 7] = np.inf
    y[5] = 0.0
    y[6, :10] = -1.0  # negative concentrations are assembled as given
    fo, Jo = oracle.assemble(m.reactants, m.products, m.k, m.row_ptr, m.col_idx, y)
    f, J = bcs.assemble(M, gpu(y), gpu(m.k))
    f1, none = bcs.assemble(M, gpu(y), gpu(m.k), J=False)
    none2, J1 = bcs.assemble(M, gpu(y), gpu(m.k), f=False)
    torch.cuda.synchronize()
    assert none is None and none2 is None
    for got, ref in ((f, fo), (J, Jo), (f1, fo), (J1, Jo)):
        assert same(got.cpu().numpy(), ref)
    f0, J0 = bcs.assemble(M, gpu(np.zeros((0, m.n))), gpu(m.k))
    torch.cuda.synchronize()
    assert f0.shape == (0, m.n) and J0.shape == (0, m.nnz)


def test_assembled_jacobian_solves_like_the_generated_one():
    """Assembly and solve chained on the device (the Newton matrix of a BDF
    step): the solve of the assembled J is bitwise the solve of the
    generator's J."""
    m, cells = config_inputs(2, ncells=5000)[0]
    M = mech_of(m)
    plan = bcs.Plan(m.row_ptr, m.col_idx)
    G, B = gpu(cells["gamma"]), gpu(cells["b"])
    _, J = bcs.assemble(M, gpu(cells["y"]), gpu(m.k), f=False)
    a = bcs.solve_batch(plan, J, G, B)
    b = bcs.solve_batch(plan, gpu(cells["values"]), G, B)
    torch.cuda.synchronize()
    for u, v in zip(a[:4], b[:4]):
        assert torch.equal(u, v)
