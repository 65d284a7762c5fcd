"""Host-side validation of mechanisms (bcs_mechanism_create): bad patterns,
species out of range and missing pattern entries are rejected before any
device call, so these run without a GPU."""
import ctypes

import numpy as np
import pytest

import paper_2405_17363_amd as bcs
from workload import gen_mechanism


def _create(n, rp, ci, reac, prod):
    L = bcs.lib()
    rp = np.ascontiguousarray(rp, np.int32)
    ci = np.ascontiguousarray(ci, np.int32)
    re = np.ascontiguousarray(np.asarray(reac).reshape(-1, 2), np.int32)
    pr = np.ascontiguousarray(np.asarray(prod).reshape(-1, 2), np.int32)
    h = ctypes.c_void_p()
    rc = L.bcs_mechanism_create(n, len(ci), rp.ctypes.data, ci.ctypes.data, re.shape[0], re.ctypes.data,
                                pr.ctypes.data, ctypes.byref(h))
    return rc, L.bcs_last_error().decode(), h


def test_missing_pattern_entry_is_rejected():
    m = gen_mechanism(30, 50)
    # drop the first off-diagonal entry of row 0 that a reaction needs
    rp, ci = m.row_ptr.copy(), m.col_idx.copy()
    q = next(q for q in range(rp[0], rp[1]) if ci[q] != 0)
    ci2 = np.delete(ci, q)
    rp2 = rp.copy()
    rp2[1:] -= 1
    rc, msg, h = _create(m.n, rp2, ci2, m.reactants, m.products)
    assert rc == -2 and "lacks" in msg and not h.value


@pytest.mark.parametrize("reac,prod,what", [
    ([[-1, -1]], [[1, -1]], "reactant"),
    ([[0, 5]], [[1, -1]], "reactant"),
    ([[0, -1]], [[7, -1]], "product"),
])
def test_species_out_of_range_are_rejected(reac, prod, what):
    n = 3
    rp = np.array([0, 3, 6, 9])
    ci = np.array([0, 1, 2] * 3)
    rc, msg, h = _create(n, rp, ci, reac, prod)
    assert rc == -1 and what in msg and not h.value


def test_malformed_pattern_is_rejected():
    rc, msg, h = _create(2, [0, 2, 3], [1, 0, 1], [[0, -1]], [[1, -1]])
    assert rc == -2 and "increasing" in msg


def test_mechanism_plan_needs_a_mechanism():
    L = bcs.lib()
    h = ctypes.c_void_p()
    assert L.bcs_plan_create_mech(None, None, ctypes.byref(h)) == -1
    assert "mechanism" in L.bcs_last_error().decode() and not h.value
