"""The entry point that allocates nothing (bcs_solve_batch_noalloc) against
bcs_solve_batch with a caller workspace: two calls in a row, the second with
a smaller batch, each bitwise equal to the workspace entry point's solve of
the same cells (same kernels, same scratch contents) and meeting the oracle's
status bar and the dense-LU bound; a batch above the scratch limit is
rejected before anything runs."""
import ctypes

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


def gpu(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def np_out(out):
    return [t.cpu().numpy() for t in out[:4]]


def test_noalloc_equals_workspace_entry_point_twice_shrinking():
    mech, cells = config_inputs(2, ncells=6000)[0]
    rp, ci = mech.row_ptr, mech.col_idx
    plan = bcs.Plan(rp, ci)
    for C in (6000, 1500):  # the second call on a smaller batch reuses the scratch
        V, G, B = gpu(cells["values"][:C]), gpu(cells["gamma"][:C]), gpu(cells["b"][:C])
        ref = np_out(bcs.solve_batch(plan, V, G, B, RTOL, 200))
        # outputs pre-filled with garbage, so stale values would show
        out = (torch.full((C, mech.n), np.nan, dtype=torch.float64, device="cuda"),
               torch.full((C,), -7, dtype=torch.int32, device="cuda"),
               torch.full((C,), np.nan, dtype=torch.float64, device="cuda"),
               torch.full((C,), -7, dtype=torch.int32, device="cuda"), None)
        got = np_out(bcs.solve_batch_noalloc(plan, V, G, B, RTOL, 200, out=out))
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            assert np.array_equal(a, b)
        x, it, res, st = got
        xo, ito, reso, sto = oracle.solve_batch(rp, ci, cells["values"][:C], cells["gamma"][:C],
                                                cells["b"][:C], precond=1)
        assert np.mean(st == sto) >= 0.99
        assert np.all(res[st == 0] <= RTOL)
        rep = lu_check(rp, ci, cells["values"][:C], cells["gamma"][:C], cells["b"][:C], x, res, st,
                       np.arange(0, C, 20))
        assert rep["checked"] >= 0.95 * len(range(0, C, 20))


def test_noalloc_rejects_batches_beyond_the_scratch():
    mech, cells = config_inputs(1, ncells=4)[0]
    plan = bcs.Plan(mech.row_ptr, mech.col_idx)
    V, G, B = gpu(cells["values"]), gpu(cells["gamma"]), gpu(cells["b"])
    x = torch.zeros((4, mech.n), dtype=torch.float64, device="cuda")
    i4 = torch.zeros(4, dtype=torch.int32, device="cuda")
    r8 = torch.zeros(4, dtype=torch.float64, device="cuda")
    L = bcs.lib()
    big = bcs.NOALLOC_MAX_CELLS + 1
    # the size check comes before any pointer is used or anything launched
    rc = L.bcs_solve_batch_noalloc(plan.handle, big, V.data_ptr(), G.data_ptr(), 1, B.data_ptr(), None, RTOL, 200,
                                   x.data_ptr(), i4.data_ptr(), r8.data_ptr(), i4.data_ptr(), None,
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -3  # BCS_ERR_UNSUPPORTED
    assert b"no-allocation" in L.bcs_last_error()
    # the largest batch the scratch holds is accepted by the size check
    assert plan.workspace_bytes(bcs.NOALLOC_MAX_CELLS) <= bcs.NOALLOC_MAX_BYTES
    assert plan.workspace_bytes(bcs.NOALLOC_MAX_CELLS + 1) > bcs.NOALLOC_MAX_BYTES
    torch.cuda.synchronize()
