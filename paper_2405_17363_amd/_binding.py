"""ctypes binding of libbcs.so: argument marshalling only."""
from __future__ import annotations

import ctypes
import glob
import os
import re
import threading
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libbcs.so")
_HEADER = os.path.join(os.path.dirname(_HERE), "include", "bcs.h")

BCS_OK = 0
BCS_CONVERGED, BCS_MAXIT, BCS_BREAKDOWN, BCS_NONFINITE = 0, 1, 2, 3
BCS_FP64, BCS_FP32_REFINE = 0, 1
BCS_PRECOND_NONE, BCS_PRECOND_JACOBI, BCS_PRECOND_ILU0 = 0, 1, 2
BCS_J_GAMMA, BCS_A_DIRECT = 0, 1
BCS_SCHED_SPAN, BCS_SCHED_DIAG = 1, 2
BCS_PART_A, BCS_PART_AT, BCS_PART_LOWER, BCS_PART_UPPER = 0, 1, 2, 3
BCS_BUDGET_INNER, BCS_BUDGET_CELL = 0, 1
BCS_GRAD_A, BCS_GRAD_VALUES = 0, 1
NOALLOC_MAX_BYTES = 4 << 20  # BCS_NOALLOC_MAX_BYTES
NOALLOC_MAX_CELLS = (NOALLOC_MAX_BYTES - 1280) // 4

_PRECOND = {"none": BCS_PRECOND_NONE, "jacobi": BCS_PRECOND_JACOBI, "ilu0": BCS_PRECOND_ILU0}
_PRECISION = {"fp64": BCS_FP64, "fp32_refine": BCS_FP32_REFINE}
_KIND = {"j_gamma": BCS_J_GAMMA, "a_direct": BCS_A_DIRECT}
_BUDGET = {"inner": BCS_BUDGET_INNER, "cell": BCS_BUDGET_CELL}
_GRAD = {"A": BCS_GRAD_A, "values": BCS_GRAD_VALUES}


class BcsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bcs error {code}: {msg}")
        self.code = code


class _Options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("precond", ctypes.c_int32),
        ("matrix_kind", ctypes.c_int32),
        ("lanes_per_cell", ctypes.c_int32),
        ("residual_replacement", ctypes.c_int32),
        ("breakdown_restarts", ctypes.c_int32),
        ("inner_rtol", ctypes.c_double),
        ("max_refine", ctypes.c_int32),
        ("jit", ctypes.c_int32),
        ("autotune", ctypes.c_int32),
        ("cell_order", ctypes.c_int32),
        ("shared_scalars", ctypes.c_int32),
        ("refine_budget", ctypes.c_int32),
        ("ilu_sweeps", ctypes.c_int32),
        ("waves_per_group", ctypes.c_int32),
    ]


_lock = threading.Lock()
_lib = None


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load libbcs.so (building it first if it does not exist)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            from . import build as _build

            _build.build()
        L = ctypes.CDLL(_LIB_PATH)
        P, I32, I64, D, VP = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        L.bcs_options_default.argtypes = [ctypes.POINTER(_Options)]
        L.bcs_options_default.restype = None
        L.bcs_plan_create.argtypes = [I32, I32, P, P, ctypes.POINTER(_Options), ctypes.POINTER(ctypes.c_void_p)]
        L.bcs_plan_create.restype = ctypes.c_int
        L.bcs_plan_destroy.argtypes = [P]
        L.bcs_plan_destroy.restype = None
        L.bcs_plan_autotune.argtypes = [P, I64, P, P, I64, P, D, I32, P, P, P, P, P]
        L.bcs_plan_autotune.restype = ctypes.c_int
        L.bcs_plan_info.argtypes = [P, P, P, P, P]
        L.bcs_plan_info.restype = ctypes.c_int
        SZ = ctypes.c_size_t
        L.bcs_workspace_bytes.argtypes = [P, I64]
        L.bcs_workspace_bytes.restype = SZ
        L.bcs_solve_batch.argtypes = [P, I64, P, P, I64, P, P, D, I32, P, P, P, P, P, P, SZ, VP]
        L.bcs_solve_batch.restype = ctypes.c_int
        L.bcs_solve_batch_noalloc.argtypes = [P, I64, P, P, I64, P, P, D, I32, P, P, P, P, P, VP]
        L.bcs_solve_batch_noalloc.restype = ctypes.c_int
        L.bcs_solve_batch_adjoint.argtypes = [P, I64, P, P, I64, P, P, D, I32, I32, P, P, P, P, P, P, P, SZ, VP]
        L.bcs_solve_batch_adjoint.restype = ctypes.c_int
        L.bcs_multi_workspace_bytes.argtypes = [I32, P, P]
        L.bcs_multi_workspace_bytes.restype = SZ
        L.bcs_solve_multi.argtypes = [I32, P, P, P, P, P, P, D, I32, P, P, P, P, P, SZ, VP]
        L.bcs_solve_multi.restype = ctypes.c_int
        L.bcs_multi_autotune.argtypes = [I32, P, P, P, P, P, P, D, I32, P, P, P, P, P]
        L.bcs_multi_autotune.restype = ctypes.c_int
        L.bcs_schedule_describe.argtypes = [I32, I32, P, P, I32, I32, I32, P, P, P, P, P, P, P]
        L.bcs_schedule_describe.restype = ctypes.c_int
        L.bcs_ilu_describe.argtypes = [I32, I32, P, P, I32, P, P, P, P]
        L.bcs_ilu_describe.restype = ctypes.c_int
        L.bcs_mechanism_create.argtypes = [I32, I32, P, P, I32, P, P, ctypes.POINTER(ctypes.c_void_p)]
        L.bcs_mechanism_create.restype = ctypes.c_int
        L.bcs_mechanism_destroy.argtypes = [P]
        L.bcs_mechanism_destroy.restype = None
        L.bcs_assemble.argtypes = [P, I64, P, P, I64, P, P, VP]
        L.bcs_assemble.restype = ctypes.c_int
        L.bcs_probe_threads_per_block.argtypes = []
        L.bcs_probe_threads_per_block.restype = ctypes.c_int
        L.bcs_probe_copy.argtypes = [P, P, I64, I32, VP]
        L.bcs_probe_copy.restype = D
        L.bcs_probe_lds.argtypes = [P, I64, I32, I32, VP]
        L.bcs_probe_lds.restype = D
        L.bcs_probe_fma.argtypes = [P, I64, I32, I32, VP]
        L.bcs_probe_fma.restype = D
        L.bcs_plan_create_mech.argtypes = [P, ctypes.POINTER(_Options), ctypes.POINTER(ctypes.c_void_p)]
        L.bcs_plan_create_mech.restype = ctypes.c_int
        L.bcs_solve_batch_mech.argtypes = [P, I64, P, P, I64, P, I64, P, P, D, I32, P, P, P, P, P, SZ, VP]
        L.bcs_solve_batch_mech.restype = ctypes.c_int
        L.bcs_debug_count_visits.argtypes = [P]
        L.bcs_debug_count_visits.restype = None
        L.bcs_last_error.argtypes = []
        L.bcs_last_error.restype = ctypes.c_char_p
        _lib = L
        return L


def exported_symbols() -> list:
    """Function names declared in the headers under include/ (bcs.h, bcs_probe.h)."""
    names = set()
    for path in sorted(glob.glob(os.path.join(os.path.dirname(_HEADER), "*.h"))):
        with open(path) as f:
            names |= set(re.findall(r"\b(bcs_[a-z_0-9]+)\s*\(", f.read()))
    return sorted(names)


def schedule_describe(row_ptr, col_idx, lanes: int, transpose=False,
                      shapes: int = BCS_SCHED_SPAN | BCS_SCHED_DIAG) -> dict:
    """The specialised kernels' gather schedule for a pattern (host only; see
    bcs_schedule_describe in include/bcs.h): steps, rows_per_lane, shape, and
    the arrays seg [rpl], row [rpl, lanes], pos [steps, lanes], col [steps, lanes].
    transpose: False/True (A, A^T) or a BCS_PART_* value (the ILU(0) triangles)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    n, nnz = rp.size - 1, ci.size
    v = [ctypes.c_int32() for _ in range(3)]
    args = (n, nnz, rp.ctypes.data, ci.ctypes.data, int(lanes), int(transpose), int(shapes))
    _check(lib().bcs_schedule_describe(*args, *[ctypes.byref(x) for x in v], None, None, None, None))
    steps, rpl, shape = (x.value for x in v)
    seg = np.zeros(rpl, np.int32)
    row = np.zeros((rpl, lanes), np.int16)
    pos = np.zeros((steps, lanes), np.int32)
    col = np.zeros((steps, lanes), np.uint8)
    _check(lib().bcs_schedule_describe(*args, None, None, None, seg.ctypes.data, row.ctypes.data, pos.ctypes.data,
                                       col.ctypes.data))
    return dict(steps=steps, rows_per_lane=rpl, shape=shape, seg=seg, row=row, pos=pos, col=col)


def ilu_describe(row_ptr, col_idx, lanes: int) -> dict:
    """The ILU(0) kernel's factorisation program for a pattern (host only; see
    bcs_ilu_describe in include/bcs.h): widths [nsteps] and words [nwords]."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    n, nnz = rp.size - 1, ci.size
    ns, nw = ctypes.c_int32(), ctypes.c_int32()
    args = (n, nnz, rp.ctypes.data, ci.ctypes.data, int(lanes))
    _check(lib().bcs_ilu_describe(*args, ctypes.byref(ns), None, ctypes.byref(nw), None))
    widths = np.zeros(ns.value, np.int32)
    words = np.zeros(nw.value, np.uint32)
    _check(lib().bcs_ilu_describe(*args, None, widths.ctypes.data, None, words.ctypes.data))
    return dict(widths=widths, words=words)


def _check(rc: int) -> None:
    if rc != BCS_OK:
        raise BcsError(rc, lib().bcs_last_error().decode())


def _torch():
    import torch

    return torch


def _stream_handle():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, name, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on a GPU device")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


class Plan:
    """A shared CSR pattern plus solver options (bcs_plan_create)."""

    def __init__(self, row_ptr, col_idx, precond: str = "jacobi", precision: str = "fp64",
                 matrix_kind: str = "j_gamma", lanes_per_cell: int = 0, residual_replacement: bool = True,
                 breakdown_restarts: int = 1, inner_rtol: float = 1e-4, max_refine: int = 10,
                 jit: bool = True, autotune: bool = True, cell_order: bool = True,
                 shared_scalars: bool = False, refine_budget: str = "inner", ilu_sweeps: int = 0,
                 waves_per_group: int = 0):
        L = lib()
        rp = np.ascontiguousarray(np.asarray(row_ptr), dtype=np.int32)
        ci = np.ascontiguousarray(np.asarray(col_idx), dtype=np.int32)
        self.n = int(rp.shape[0] - 1)
        self.nnz = int(ci.shape[0])
        self.row_ptr, self.col_idx = rp, ci
        opt = _Options()
        L.bcs_options_default(ctypes.byref(opt))
        opt.precision = _PRECISION[precision]
        opt.precond = _PRECOND[precond]
        opt.matrix_kind = _KIND[matrix_kind]
        opt.lanes_per_cell = int(lanes_per_cell)
        opt.residual_replacement = int(bool(residual_replacement))
        opt.breakdown_restarts = int(breakdown_restarts)
        opt.inner_rtol = float(inner_rtol)
        opt.max_refine = int(max_refine)
        opt.jit = int(bool(jit))
        opt.autotune = int(bool(autotune))
        opt.cell_order = int(bool(cell_order))
        opt.shared_scalars = int(bool(shared_scalars))
        opt.refine_budget = _BUDGET[refine_budget]
        opt.ilu_sweeps = int(ilu_sweeps)
        opt.waves_per_group = int(waves_per_group)
        self.options = opt
        self.precision, self.precond, self.matrix_kind = precision, precond, matrix_kind
        h = ctypes.c_void_p()
        rc = L.bcs_plan_create(self.n, self.nnz, rp.ctypes.data, ci.ctypes.data if self.nnz else None,
                               ctypes.byref(opt), ctypes.byref(h))
        self._h = None
        _check(rc)
        self._h = h

    @classmethod
    def from_mechanism(cls, mech: "Mechanism", precond: str = "jacobi", lanes_per_cell: int = 0,
                       autotune: bool = True, cell_order: bool = True, residual_replacement: bool = True,
                       breakdown_restarts: int = 1):
        """A plan for the mechanism's pattern whose solve_batch_mech assembles
        each cell's J inside the solve (bcs_plan_create_mech).  The plan keeps
        a reference to the mechanism."""
        L = lib()
        self = cls.__new__(cls)
        self.n, self.nnz = mech.n, mech.nnz
        self.row_ptr, self.col_idx = mech.row_ptr, mech.col_idx
        opt = _Options()
        L.bcs_options_default(ctypes.byref(opt))
        opt.precond = _PRECOND[precond]
        opt.lanes_per_cell = int(lanes_per_cell)
        opt.autotune = int(bool(autotune))
        opt.cell_order = int(bool(cell_order))
        opt.residual_replacement = int(bool(residual_replacement))
        opt.breakdown_restarts = int(breakdown_restarts)
        self.options = opt
        self.precision, self.precond, self.matrix_kind = "fp64", precond, "j_gamma"
        self.mechanism = mech
        h = ctypes.c_void_p()
        self._h = None
        _check(L.bcs_plan_create_mech(mech.handle, ctypes.byref(opt), ctypes.byref(h)))
        self._h = h
        return self

    @property
    def handle(self):
        return self._h

    def workspace_bytes(self, ncells: int) -> int:
        return int(lib().bcs_workspace_bytes(self._h, int(ncells)))

    def workspace(self, ncells: int, device=None):
        """A device workspace for a solve of `ncells` cells (a uint8 tensor)."""
        return _workspace(self.workspace_bytes(ncells), device)

    def info(self) -> dict:
        v = [ctypes.c_int32() for _ in range(4)]
        _check(lib().bcs_plan_info(self._h, *[ctypes.byref(x) for x in v]))
        return dict(lanes_per_cell=v[0].value, rows_per_lane=v[1].value, steps_per_lane=v[2].value,
                    cells_per_wg=v[3].value, jit=bool(self.options.jit))

    def autotune(self, values, gamma, b, rtol: float = 1e-10, maxit: int = 200) -> int:
        """Time every lanes-per-cell layout on this batch and keep the fastest; returns lanes per cell."""
        torch = _torch()
        values = _dev(values, torch.float64, "values", (values.shape[0], self.nnz))
        C = values.shape[0]
        _dev(b, torch.float64, "b", (C, self.n))
        g, gs = _gamma_arg(gamma, C, values.device)
        x = torch.empty((C, self.n), dtype=torch.float64, device=values.device)
        it = torch.empty(C, dtype=torch.int32, device=values.device)
        rs = torch.empty(C, dtype=torch.float64, device=values.device)
        st = torch.empty(C, dtype=torch.int32, device=values.device)
        lanes = ctypes.c_int32()
        torch.cuda.synchronize()
        _check(lib().bcs_plan_autotune(self._h, C, values.data_ptr(), g.data_ptr(), gs, b.data_ptr(), float(rtol),
                                       int(maxit), x.data_ptr(), it.data_ptr(), rs.data_ptr(), st.data_ptr(),
                                       ctypes.byref(lanes)))
        return lanes.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.bcs_plan_destroy(h)
            self._h = None


def _gamma_arg(gamma, ncells, device):
    torch = _torch()
    if not isinstance(gamma, torch.Tensor):
        gamma = torch.tensor([float(gamma)], dtype=torch.float64, device=device)
    _dev(gamma, torch.float64, "gamma")
    if gamma.numel() == 1:
        return gamma, 0
    if gamma.numel() != ncells:
        raise ValueError("gamma must have 1 or ncells elements")
    return gamma, 1


def _workspace(nbytes: int, device):
    torch = _torch()
    ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    if ws.data_ptr() % 256:
        raise RuntimeError("the device allocator returned a workspace that is not 256-byte aligned")
    return ws


def _check_ws(ws, need: int, device):
    torch = _torch()
    if ws is None:
        return _workspace(need, device)
    _dev(ws, torch.uint8, "workspace")
    if ws.numel() < need:
        raise ValueError(f"workspace holds {ws.numel()} bytes, {need} needed")
    return ws


def solve_batch(plan: Plan, values, gamma, b, rtol: float = 1e-10, maxit: int = 200, out=None, x0=None,
                workspace=None):
    """Solve every cell's system; returns (x, iters, resid, status, refinements).

    x0: optional initial guess [ncells, n] (may be the `x` of `out`); workspace:
    optional uint8 device tensor of at least plan.workspace_bytes(ncells) bytes
    (one is allocated through torch's caching allocator otherwise)."""
    torch = _torch()
    values = _dev(values, torch.float64, "values")
    ncells = values.shape[0] if values.dim() == 2 else 0
    _dev(values, torch.float64, "values", (ncells, plan.nnz))
    _dev(b, torch.float64, "b", (ncells, plan.n))
    if x0 is not None:
        _dev(x0, torch.float64, "x0", (ncells, plan.n))
    g, gs = _gamma_arg(gamma, ncells, values.device)
    ws = _check_ws(workspace, plan.workspace_bytes(ncells), values.device)
    if out is None:
        x = torch.empty((ncells, plan.n), dtype=torch.float64, device=values.device)
        iters = torch.empty(ncells, dtype=torch.int32, device=values.device)
        resid = torch.empty(ncells, dtype=torch.float64, device=values.device)
        status = torch.empty(ncells, dtype=torch.int32, device=values.device)
        refin = torch.empty(ncells, dtype=torch.int32, device=values.device)
    else:
        x, iters, resid, status, refin = out
    rc = lib().bcs_solve_batch(plan.handle, ncells, values.data_ptr(), g.data_ptr(), gs, b.data_ptr(),
                               x0.data_ptr() if x0 is not None else None, float(rtol), int(maxit), x.data_ptr(),
                               iters.data_ptr(), resid.data_ptr(), status.data_ptr(),
                               refin.data_ptr() if refin is not None else None, ws.data_ptr(), ws.numel(),
                               _stream_handle())
    _check(rc)
    return x, iters, resid, status, refin


def solve_batch_noalloc(plan: Plan, values, gamma, b, rtol: float = 1e-10, maxit: int = 200, out=None, x0=None):
    """solve_batch without a workspace (bcs_solve_batch_noalloc): the solve's
    scratch is the library's own device array (at most NOALLOC_MAX_CELLS
    cells).  Calls that overlap on one GPU race.  With `out` given (x, iters,
    resid, status, refinements or None) nothing at all is allocated."""
    torch = _torch()
    values = _dev(values, torch.float64, "values")
    ncells = values.shape[0] if values.dim() == 2 else 0
    _dev(values, torch.float64, "values", (ncells, plan.nnz))
    _dev(b, torch.float64, "b", (ncells, plan.n))
    if x0 is not None:
        _dev(x0, torch.float64, "x0", (ncells, plan.n))
    g, gs = _gamma_arg(gamma, ncells, values.device)
    if out is None:
        x = torch.empty((ncells, plan.n), dtype=torch.float64, device=values.device)
        iters = torch.empty(ncells, dtype=torch.int32, device=values.device)
        resid = torch.empty(ncells, dtype=torch.float64, device=values.device)
        status = torch.empty(ncells, dtype=torch.int32, device=values.device)
        refin = torch.empty(ncells, dtype=torch.int32, device=values.device)
    else:
        x, iters, resid, status, refin = out
    rc = lib().bcs_solve_batch_noalloc(plan.handle, ncells, values.data_ptr(), g.data_ptr(), gs, b.data_ptr(),
                                       x0.data_ptr() if x0 is not None else None, float(rtol), int(maxit),
                                       x.data_ptr(), iters.data_ptr(), resid.data_ptr(), status.data_ptr(),
                                       refin.data_ptr() if refin is not None else None, _stream_handle())
    _check(rc)
    return x, iters, resid, status, refin


def solve_batch_mech(plan: Plan, y, k, gamma, b, rtol: float = 1e-10, maxit: int = 200, out=None, x0=None,
                     workspace=None):
    """Solve every cell's Newton system with J assembled from its
    concentrations inside the solve (bcs_solve_batch_mech); plan from
    Plan.from_mechanism.  y: [C, n]; k: [R] (shared) or [C, R]; returns (x,
    iters, resid, status)."""
    torch = _torch()
    mech = getattr(plan, "mechanism", None)
    if mech is None:
        raise ValueError("the plan was not made by Plan.from_mechanism")
    y = _dev(y, torch.float64, "y")
    ncells = y.shape[0] if y.dim() == 2 else 0
    _dev(y, torch.float64, "y", (ncells, plan.n))
    _dev(b, torch.float64, "b", (ncells, plan.n))
    k = _dev(k, torch.float64, "k")
    if k.dim() == 1:
        _dev(k, torch.float64, "k", (mech.R,))
        ks = 0
    else:
        _dev(k, torch.float64, "k", (ncells, mech.R))
        ks = mech.R
    if x0 is not None:
        _dev(x0, torch.float64, "x0", (ncells, plan.n))
    g, gs = _gamma_arg(gamma, ncells, y.device)
    ws = _check_ws(workspace, plan.workspace_bytes(ncells), y.device)
    if out is None:
        x = torch.empty((ncells, plan.n), dtype=torch.float64, device=y.device)
        iters = torch.empty(ncells, dtype=torch.int32, device=y.device)
        resid = torch.empty(ncells, dtype=torch.float64, device=y.device)
        status = torch.empty(ncells, dtype=torch.int32, device=y.device)
    else:
        x, iters, resid, status = out[:4]
    _check(lib().bcs_solve_batch_mech(plan.handle, ncells, y.data_ptr(), k.data_ptr(), ks, g.data_ptr(), gs,
                                      b.data_ptr(), x0.data_ptr() if x0 is not None else None, float(rtol),
                                      int(maxit), x.data_ptr(), iters.data_ptr(), resid.data_ptr(),
                                      status.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle()))
    return x, iters, resid, status


def solve_batch_adjoint(plan: Plan, values, gamma, x, g, rtol: float = 1e-10, maxit: int = 200,
                        grad_kind: str = "A", grad_gamma: bool = False, workspace=None):
    """Adjoint solve: returns (grad_b = lambda, grad_vals, grad_gamma, iters, resid, status).

    grad_kind "A": grad_vals = dL/dA on the pattern; "values": dL/d(values)
    (dL/dJ in J mode).  grad_gamma: also return dL/dgamma per cell (J mode),
    else None."""
    torch = _torch()
    values = _dev(values, torch.float64, "values")
    ncells = values.shape[0]
    _dev(x, torch.float64, "x", (ncells, plan.n))
    _dev(g, torch.float64, "g", (ncells, plan.n))
    gm, gs = _gamma_arg(gamma, ncells, values.device)
    dev = values.device
    ws = _check_ws(workspace, plan.workspace_bytes(ncells), dev)
    grad_b = torch.empty((ncells, plan.n), dtype=torch.float64, device=dev)
    grad_v = torch.empty((ncells, plan.nnz), dtype=torch.float64, device=dev)
    grad_g = torch.empty(ncells, dtype=torch.float64, device=dev) if grad_gamma else None
    iters = torch.empty(ncells, dtype=torch.int32, device=dev)
    resid = torch.empty(ncells, dtype=torch.float64, device=dev)
    status = torch.empty(ncells, dtype=torch.int32, device=dev)
    rc = lib().bcs_solve_batch_adjoint(plan.handle, ncells, values.data_ptr(), gm.data_ptr(), gs, x.data_ptr(),
                                       g.data_ptr(), float(rtol), int(maxit), _GRAD[grad_kind], grad_b.data_ptr(),
                                       grad_v.data_ptr(), grad_g.data_ptr() if grad_g is not None else None,
                                       iters.data_ptr(), resid.data_ptr(), status.data_ptr(), ws.data_ptr(),
                                       ws.numel(), _stream_handle())
    _check(rc)
    return grad_b, grad_v, grad_g, iters, resid, status


def _multi_args(plans: Sequence[Plan], values: Sequence, gammas: Sequence, bs: Sequence):
    """Pointer arrays of the one-launch form and the output tensors they point to."""
    torch = _torch()
    m = len(plans)
    outs = []
    arrs = {k: (ctypes.c_void_p * m)() for k in ("plans", "values", "gamma", "b", "x", "iters", "resid", "status")}
    nc = (ctypes.c_int64 * m)()
    gst = (ctypes.c_int64 * m)()
    keep = []
    for i, (pl, v, g, b) in enumerate(zip(plans, values, gammas, bs)):
        _dev(v, torch.float64, "values")
        C = v.shape[0]
        _dev(v, torch.float64, "values", (C, pl.nnz))
        _dev(b, torch.float64, "b", (C, pl.n))
        gg, gs = _gamma_arg(g, C, v.device)
        keep.append(gg)
        x = torch.empty((C, pl.n), dtype=torch.float64, device=v.device)
        it = torch.empty(C, dtype=torch.int32, device=v.device)
        rs = torch.empty(C, dtype=torch.float64, device=v.device)
        st = torch.empty(C, dtype=torch.int32, device=v.device)
        outs.append((x, it, rs, st))
        nc[i] = C
        gst[i] = gs
        for k, t in (("values", v), ("gamma", gg), ("b", b), ("x", x), ("iters", it), ("resid", rs),
                     ("status", st)):
            arrs[k][i] = t.data_ptr()
        arrs["plans"][i] = pl.handle.value
    return m, arrs, nc, gst, outs, keep


def solve_multi(plans: Sequence[Plan], values: Sequence, gammas: Sequence, bs: Sequence, rtol: float = 1e-10,
                maxit: int = 200, workspace=None):
    """One persistent launch over several mechanisms; per mechanism (x, iters, resid, status)."""
    m, arrs, nc, gst, outs, keep = _multi_args(plans, values, gammas, bs)  # keep: tensors alive across the call
    need = int(lib().bcs_multi_workspace_bytes(m, arrs["plans"], nc))
    ws = _check_ws(workspace, need, values[0].device)
    rc = lib().bcs_solve_multi(m, arrs["plans"], nc, arrs["values"], arrs["gamma"], gst, arrs["b"], float(rtol),
                               int(maxit), arrs["x"], arrs["iters"], arrs["resid"], arrs["status"], ws.data_ptr(),
                               ws.numel(), _stream_handle())
    _check(rc)
    return outs


def multi_autotune(plans: Sequence[Plan], values: Sequence, gammas: Sequence, bs: Sequence, rtol: float = 1e-10,
                   maxit: int = 200) -> list:
    """Choose every plan's lanes per cell for the one-launch form by timing it on these batches.

    The choice stays in the plans (their adjoint kernels follow it); returns the lane counts.
    Synchronises the device.
    """
    m, arrs, nc, gst, outs, keep = _multi_args(plans, values, gammas, bs)  # keep: tensors alive across the call
    lanes = (ctypes.c_int32 * m)()
    _check(lib().bcs_multi_autotune(m, arrs["plans"], nc, arrs["values"], arrs["gamma"], gst, arrs["b"],
                                    float(rtol), int(maxit), arrs["x"], arrs["iters"], arrs["resid"],
                                    arrs["status"], lanes))
    return list(lanes)


class Mechanism:
    """A mass-action mechanism on a CSR pattern (bcs_mechanism_create): the
    gather tables of its rates f and Jacobian J, on the current device."""

    def __init__(self, n: int, reactants, products, row_ptr, col_idx):
        L = lib()
        rp = np.ascontiguousarray(np.asarray(row_ptr), dtype=np.int32)
        ci = np.ascontiguousarray(np.asarray(col_idx), dtype=np.int32)
        re = np.ascontiguousarray(np.asarray(reactants).reshape(-1, 2), dtype=np.int32)
        pr = np.ascontiguousarray(np.asarray(products).reshape(-1, 2), dtype=np.int32)
        if re.shape != pr.shape:
            raise ValueError("reactants and products must both have shape [R, 2]")
        self.n, self.nnz, self.R = int(n), int(ci.shape[0]), int(re.shape[0])
        self.row_ptr, self.col_idx = rp, ci
        if rp.shape[0] != self.n + 1:
            raise ValueError("row_ptr must have n + 1 entries")
        h = ctypes.c_void_p()
        self._h = None
        _check(L.bcs_mechanism_create(self.n, self.nnz, rp.ctypes.data, ci.ctypes.data, self.R, re.ctypes.data,
                                      pr.ctypes.data, ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.bcs_mechanism_destroy(h)
            self._h = None


def assemble(mech: Mechanism, y, k, f: bool = True, J: bool = True, out=None):
    """Mass-action rates and Jacobian of every cell (bcs_assemble): returns
    (f [C, n] or None, J [C, nnz] or None).  y: [C, n] FP64 device tensor;
    k: [R] (shared) or [C, R] (per cell) FP64 device tensor; out: optional
    (f, J) tensors to write into."""
    torch = _torch()
    y = _dev(y, torch.float64, "y")
    C = y.shape[0] if y.dim() == 2 else 0
    _dev(y, torch.float64, "y", (C, mech.n))
    k = _dev(k, torch.float64, "k")
    if k.dim() == 1:
        _dev(k, torch.float64, "k", (mech.R,))
        ks = 0
    else:
        _dev(k, torch.float64, "k", (C, mech.R))
        ks = mech.R
    if out is not None:
        fo, Jo = out
    else:
        fo = torch.empty((C, mech.n), dtype=torch.float64, device=y.device) if f else None
        Jo = torch.empty((C, mech.nnz), dtype=torch.float64, device=y.device) if J else None
    if fo is not None:
        _dev(fo, torch.float64, "f", (C, mech.n))
    if Jo is not None:
        _dev(Jo, torch.float64, "J", (C, mech.nnz))
    _check(lib().bcs_assemble(mech.handle, C, y.data_ptr(), k.data_ptr(), ks,
                              fo.data_ptr() if fo is not None else None, Jo.data_ptr() if Jo is not None else None,
                              _stream_handle()))
    return fo, Jo


class BatchedSolveWarning(UserWarning):
    """Cells of a differentiable solve whose forward or adjoint solve did not converge."""


class BatchedSolve:
    """Differentiable batched solve x = (I - gamma J)^-1 b (J mode) or A^-1 b.

    ``BatchedSolve.apply(values, gamma, b, plan, rtol, maxit)`` returns
    ``(x, status)``: x differentiable, status the per-cell int32 solve status
    (not differentiable; cells with status != 0 carry the solver's best
    iterate, not the solution).  Backward runs the library's adjoint solve
    (transposed BiCGStab), whose epilogue writes the gradients with respect to
    the inputs themselves (dL/dJ and dL/dgamma in J mode, dL/dA in A mode);
    cells whose adjoint solve did not converge are reported with a
    BatchedSolveWarning.  A scalar gamma tensor is expanded to one value per
    cell, so autograd sums the per-cell gamma gradients.
    """

    _fn = None

    @classmethod
    def _function(cls):
        if cls._fn is None:
            torch = _torch()

            class _F(torch.autograd.Function):
                @staticmethod
                def forward(ctx, values, gamma, b, plan, rtol=1e-10, maxit=200):
                    values_c = values.contiguous()
                    x, iters, resid, status, _ = solve_batch(plan, values_c, gamma, b.contiguous(), rtol, maxit)
                    ctx.plan, ctx.rtol, ctx.maxit = plan, rtol, maxit
                    ctx.save_for_backward(values_c, gamma if isinstance(gamma, torch.Tensor) else None, x)
                    ctx.gamma_obj = gamma
                    ctx.mark_non_differentiable(status)
                    return x, status

                @staticmethod
                def backward(ctx, gx, _gstatus):
                    values, gamma_t, x = ctx.saved_tensors
                    plan = ctx.plan
                    gamma = gamma_t if gamma_t is not None else ctx.gamma_obj
                    j_mode = plan.matrix_kind != "a_direct"
                    want_g = j_mode and gamma_t is not None and ctx.needs_input_grad[1]
                    grad_b, grad_v, grad_g, _, _, st = solve_batch_adjoint(
                        plan, values, gamma, x, gx.contiguous(), ctx.rtol, ctx.maxit, grad_kind="values",
                        grad_gamma=want_g)
                    bad = int((st != BCS_CONVERGED).sum().item())
                    if bad:
                        import warnings

                        warnings.warn(f"{bad} of {st.numel()} cells: the adjoint solve did not converge; their "
                                      "gradients come from the best iterate", BatchedSolveWarning, stacklevel=2)
                    return grad_v, grad_g, grad_b, None, None, None

            cls._fn = _F
        return cls._fn

    @classmethod
    def apply(cls, values, gamma, b, plan, rtol=1e-10, maxit=200):
        torch = _torch()
        if isinstance(gamma, torch.Tensor) and gamma.numel() == 1 and values.dim() == 2 and values.shape[0] > 1:
            gamma = gamma.reshape(1).expand(values.shape[0]).contiguous()
        return cls._function().apply(values, gamma, b, plan, rtol, maxit)
