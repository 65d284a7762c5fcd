"""The C-ABI library loads, exports every declared symbol, and rejects bad
patterns and options before touching a device (runs without a GPU)."""
import ctypes

import numpy as np
import pytest

import paper_2405_17363_amd as bcs
from paper_2405_17363_amd._binding import _Options


def test_library_exports_every_declared_symbol():
    L = bcs.lib()
    names = bcs.exported_symbols()
    assert {"bcs_plan_create", "bcs_solve_batch", "bcs_solve_batch_adjoint", "bcs_solve_multi",
            "bcs_multi_autotune", "bcs_last_error", "bcs_plan_destroy", "bcs_options_default",
            "bcs_plan_info"} <= set(names)
    for name in names:
        assert hasattr(L, name), name


def test_options_struct_layout_and_defaults():
    L = bcs.lib()
    o = _Options()
    L.bcs_options_default(ctypes.byref(o))
    assert o.precision == bcs.BCS_FP64 and o.precond == 1 and o.matrix_kind == bcs.BCS_J_GAMMA
    assert o.residual_replacement == 1 and o.breakdown_restarts == 1
    assert o.inner_rtol == 1e-4 and o.max_refine == 10
    assert o.jit == 1 and o.autotune == 1 and o.cell_order == 1 and o.shared_scalars == 0
    assert o.refine_budget == bcs.BCS_BUDGET_INNER
    assert ctypes.sizeof(_Options) == 64


def _create(rp, ci, **kw):
    L = bcs.lib()
    o = _Options()
    L.bcs_options_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    rp = np.asarray(rp, np.int32)
    ci = np.asarray(ci, np.int32)
    h = ctypes.c_void_p()
    rc = L.bcs_plan_create(len(rp) - 1, len(ci), rp.ctypes.data, ci.ctypes.data, ctypes.byref(o), ctypes.byref(h))
    return rc, L.bcs_last_error().decode(), h


@pytest.mark.parametrize("rp,ci,what", [
    ([1, 2, 3], [0, 1], "row_ptr[0]"),
    ([0, 2, 3], [0, 1], "row_ptr[n]"),
    ([0, 2, 1], [0], "row_ptr decreases"),
    ([0, 2, 4], [1, 0, 0, 1], "strictly increasing"),
    ([0, 2, 4], [0, 0, 0, 1], "strictly increasing"),
    ([0, 2, 4], [0, 2, 0, 1], "out of range"),
    ([0, 1, 2], [1, 0], "diagonal"),
])
def test_invalid_patterns_are_rejected(rp, ci, what):
    rc, msg, h = _create(rp, ci)
    assert rc in (-1, -2), msg
    assert what.split()[0] in msg
    assert not h.value


@pytest.mark.parametrize("field,value", [("precision", 7), ("precond", 5), ("matrix_kind", 3),
                                          ("lanes_per_cell", 8), ("residual_replacement", 2),
                                          ("breakdown_restarts", -1), ("jit", 2), ("autotune", 3), ("cell_order", 2),
                                          ("shared_scalars", 2), ("refine_budget", 2), ("waves_per_group", 3),
                                          ("waves_per_group", 16)])
def test_invalid_options_are_rejected(field, value):
    rc, msg, h = _create([0, 1, 2], [0, 1], **{field: value})
    assert rc == -1, msg
    assert not h.value


def test_missing_diagonal_allowed_without_jacobi_in_a_mode():
    # A_DIRECT + no preconditioner does not need the diagonal: validation
    # passes and only the (absent) device can stop the plan.
    rc, msg, h = _create([0, 1, 2], [1, 0], matrix_kind=1, precond=0)
    assert rc in (0, -4), msg
    if rc == 0:
        bcs.lib().bcs_plan_destroy(h)


@pytest.mark.parametrize("extra", [dict(), dict(lanes_per_cell=32, jit=0), dict(lanes_per_cell=32, precision=1)])
def test_shared_scalars_needs_fixed_lanes_fp64_and_jit(extra):
    rc, msg, h = _create([0, 1, 2], [0, 1], shared_scalars=1, **extra)
    assert rc == -1 and "shared_scalars" in msg
    assert not h.value


@pytest.mark.parametrize("extra", [dict(jit=0), dict(precision=1), dict(precond=2)])
def test_waves_per_group_needs_a_forward_fp64_kernel_compiled_per_pattern(extra):
    rc, msg, h = _create([0, 1, 2], [0, 1], waves_per_group=2, **extra)
    assert rc == -3 and "waves_per_group" in msg
    assert not h.value


def test_more_than_255_rows_is_unsupported():
    n = 256
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    rc, msg, h = _create(rp, ci)
    assert rc == -3 and "255" in msg
    assert not h.value


@pytest.mark.parametrize("nmech,null_plan", [(0, False), (9, False), (2, True)])
def test_multi_entry_points_reject_bad_counts_and_null_plans(nmech, null_plan):
    # both entry points check the mechanism count (1..8) and, for the autotuner,
    # NULL plans before any device call
    L = bcs.lib()
    m = max(nmech, 1)
    plans = (ctypes.c_void_p * m)()  # all NULL
    arrs = [(ctypes.c_void_p * m)() for _ in range(8)]
    nc = (ctypes.c_int64 * m)()
    gst = (ctypes.c_int64 * m)()
    rc = L.bcs_multi_autotune(nmech, plans, nc, arrs[0], arrs[1], gst, arrs[2], 1e-10, 200, arrs[3], arrs[4],
                              arrs[5], arrs[6], None)
    assert rc == -1, L.bcs_last_error().decode()
    msg = L.bcs_last_error().decode()
    assert ("NULL" in msg) if null_plan else ("nmech" in msg)
    if not null_plan:
        rc = L.bcs_solve_multi(nmech, plans, nc, arrs[0], arrs[1], gst, arrs[2], 1e-10, 200, arrs[3], arrs[4],
                               arrs[5], arrs[6], None, 0, None)
        assert rc == -1 and "nmech" in L.bcs_last_error().decode()
        assert L.bcs_multi_workspace_bytes(nmech, plans, nc) == 0


def test_workspace_size_needs_a_plan_and_a_cell_count():
    L = bcs.lib()
    assert L.bcs_workspace_bytes(None, 10) == 0
    assert L.bcs_workspace_bytes(None, -1) == 0


def test_solve_entry_points_reject_a_null_plan_before_any_device_call():
    L = bcs.lib()
    rc = L.bcs_solve_batch(None, 1, None, None, 0, None, None, 1e-10, 200, None, None, None, None, None, None, 0,
                           None)
    assert rc == -1 and "plan" in L.bcs_last_error().decode()
    rc = L.bcs_solve_batch_adjoint(None, 1, None, None, 0, None, None, 1e-10, 200, 0, None, None, None, None, None,
                                   None, None, 0, None)
    assert rc == -1 and "plan" in L.bcs_last_error().decode()
