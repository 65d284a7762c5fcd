"""Solves whose Jacobian is assembled inside the solve kernel from the cells'
concentrations (bcs_plan_create_mech / bcs_solve_batch_mech).

The kernel assembles J with the sums and roundings of bcs_assemble, so the
bar is bitwise equality with bcs_assemble followed by bcs_solve_batch on the
same plan (whose parity with the oracle the other GPU tests establish), on
the benchmark workload's 100,000 cells, with shared and per-cell rate
constants, with a warm start, and on all three mechanisms of the uneven
batch; plus the oracle's statuses and dense LU on a sample, and the argument
checks."""
import numpy as np
import pytest

import oracle
from parity import lu_check
from workload import config_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - collected on CPU hosts too
    pytest.skip("no GPU", allow_module_level=True)

import paper_2405_17363_amd as bcs  # noqa: E402

RTOL = 1e-10


def gpu(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def mech_of(m):
    return bcs.Mechanism(m.n, m.reactants, m.products, m.row_ptr, m.col_idx)


def both_ways(plan, M, y, k, G, B, x0=None):
    out = bcs.solve_batch_mech(plan, y, k, G, B, RTOL, 200, x0=x0)
    _, J = bcs.assemble(M, y, k, f=False)
    ref = bcs.solve_batch(plan, J, G, B, RTOL, 200, x0=x0)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out], [t.cpu().numpy() for t in ref[:4]]


def test_config3_full_size_bitwise_and_against_the_oracle():
    m, cells = config_inputs(3)[0]
    M = mech_of(m)
    plan = bcs.Plan.from_mechanism(M)
    y, k, G, B = gpu(cells["y"]), gpu(m.k), gpu(cells["gamma"]), gpu(cells["b"])
    got, ref = both_ways(plan, M, y, k, G, B)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
    x, it, res, st = got
    assert np.mean(st == 0) >= 0.99 and np.all(res[st == 0] <= RTOL)
    sample = np.random.default_rng(11).choice(100_000, 400, replace=False)
    xo, ito, reso, sto = oracle.solve_batch(m.row_ptr, m.col_idx, cells["values"][sample], cells["gamma"][sample],
                                            cells["b"][sample], precond=1)
    assert np.mean(st[sample] == sto) >= 0.98
    out = lu_check(m.row_ptr, m.col_idx, cells["values"], cells["gamma"], cells["b"], x, res, st, sample)
    assert out["checked"] >= 390


def test_per_cell_rate_constants_warm_start_and_all_mechanisms():
    for m, cells in config_inputs(4, ncells=6000):
        M = mech_of(m)
        plan = bcs.Plan.from_mechanism(M)  # n = 200: the J term program takes the LDS beyond 64 KiB
        C = cells["y"].shape[0]
        kc = m.k[None, :] * 10.0 ** np.random.default_rng(m.n).uniform(-1, 1, size=(C, m.R))
        y, G, B = gpu(cells["y"]), gpu(cells["gamma"]), gpu(cells["b"])
        for k in (gpu(m.k), gpu(kc)):
            got, ref = both_ways(plan, M, y, k, G, B)
            for a, b in zip(got, ref):
                assert np.array_equal(a, b), m.n
        x0 = gpu(0.5 * got[0])
        got, ref = both_ways(plan, M, y, gpu(kc), G, B, x0=x0)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), m.n


def test_autotune_keeps_the_mechanism_kernel_in_step():
    m, cells = config_inputs(2, ncells=4000)[0]
    M = mech_of(m)
    plan = bcs.Plan.from_mechanism(M)
    y, k, G, B = gpu(cells["y"]), gpu(m.k), gpu(cells["gamma"]), gpu(cells["b"])
    plan.autotune(gpu(cells["values"]), G, B)
    got, ref = both_ways(plan, M, y, k, G, B)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


def test_mechanism_solve_argument_checks():
    m, cells = config_inputs(1, ncells=8)[0]
    M = mech_of(m)
    plain = bcs.Plan(m.row_ptr, m.col_idx)
    y, k, G, B = gpu(cells["y"]), gpu(m.k), gpu(cells["gamma"]), gpu(cells["b"])
    with pytest.raises(ValueError):
        bcs.solve_batch_mech(plain, y, k, G, B)
    with pytest.raises(bcs.BcsError) as e:
        bcs.Plan.from_mechanism(M, precond="ilu0")
    assert e.value.code == -3
    plan = bcs.Plan.from_mechanism(M)
    x, it, res, st = bcs.solve_batch_mech(plan, gpu(np.zeros((0, m.n))), k, gpu(np.zeros(0)), gpu(np.zeros((0, m.n))))
    assert x.shape == (0, m.n)
    torch.cuda.synchronize()


def same(a, b):
    """Bitwise up to NaN payloads (signs of zero included)."""
    return np.array_equal(a, b, equal_nan=True) and np.array_equal(np.signbit(a), np.signbit(b))


@pytest.mark.parametrize("lanes", [16, 32, 64])
def test_edge_concentrations_at_every_lane_count(lanes):
    """NaN, Inf, zero and negative concentrations, and each lane count's
    layout (its padding steps take CSR position 0's value, its padding rows
    get no terms): the fused solve's outputs are bitwise those of assembly
    followed by a solve with the same plan, NaN-aware."""
    m, cells = config_inputs(1)[0]
    y = cells["y"].copy()
    y[3, 5] = np.nan
    y[4, 7] = np.inf
    y[5] = 0.0
    y[6, :10] = -1.0
    M = mech_of(m)
    plan = bcs.Plan.from_mechanism(M, lanes_per_cell=lanes)
    assert plan.info()["lanes_per_cell"] == lanes
    G, B = gpu(cells["gamma"]), gpu(cells["b"])
    for k in (gpu(m.k), gpu(m.k[None, :] * np.linspace(0.5, 2.0, y.shape[0])[:, None])):
        got, ref = both_ways(plan, M, gpu(y), k, G, B)
        for a, b in zip(got, ref):
            assert same(a, b)
