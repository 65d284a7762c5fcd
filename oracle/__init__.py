"""CPU oracle for batched (I - gamma*J) x = b solves -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It is a plain, slow, obviously correct FP64 (and, for
the mixed form, FP32) implementation in C (``oracle.c``), loaded through
ctypes.  It shares no code with the HIP library.

Functions (all take/return numpy arrays):
  solve_batch   BiCGStab per cell (FP64), optional x0      -> x, iters, resid, status
  solve_batch_f the same BiCGStab in FP32 (mixed form's inner solver)
  ilu0          ILU(0) factors of one matrix on its pattern; ilu_apply: (LU)^-1 p
  lu_batch      dense LU with partial pivoting per cell   -> x (ground truth)
  adjoint_batch lambda = A^-T g and dL/dA on the pattern   -> grad_b, grad_A, iters, resid, status
  mixed_batch   FP32 inner BiCGStab + FP64 refinement      -> x, iters, refinements, resid, status
  solve_groups  Block-cells (N): runs of cells solved as one block-diagonal system -> x, iters, resid, status
  form_a        A = I - gamma*J on the pattern
  assemble      mass-action rates f and Jacobian J per cell   -> f, J
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

CONVERGED, MAXIT, BREAKDOWN, NONFINITE = 0, 1, 2, 3
J_GAMMA, A_DIRECT = 0, 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "bicgstab_body.h")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_I = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64 = ctypes.c_int64
_int = ctypes.c_int
_dbl = ctypes.c_double


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C, OpenMP, no FMA contraction)."""
    with _lock:
        if force or not os.path.exists(_LIB_PATH):
            tmp = _LIB_PATH + ".tmp%d" % os.getpid()
            cmd = ["gcc", "-O3", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
                   "-std=c11", "-Wall", "-o", tmp, _SRC[0], "-lm"]
            subprocess.run(cmd, check=True, cwd=_HERE)
            os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # ORACLE_LIB: a separately built copy of the same source (the sanitizer
    # tests load an AddressSanitizer / UBSan build this way)
    path = os.environ.get("ORACLE_LIB") or build()
    lib = ctypes.CDLL(path)
    _vp = ctypes.c_void_p
    lib.oracle_solve_batch.argtypes = [_i64, _int, _int, _I, _I, _D, _D, _i64, _int, _D, _vp, _dbl, _int, _int,
                                       _int, _int, _int, _D, _I, _D, _I, _int]
    lib.oracle_ilu0.argtypes = [_int, _I, _I, _D, _D]
    lib.oracle_ilu0.restype = _int
    lib.oracle_ilu_apply.argtypes = [_int, _I, _I, _D, _int, _D, _D]
    lib.oracle_ilu_apply.restype = None
    lib.oracle_solve_batch.restype = None
    lib.oracle_lu_batch.argtypes = [_i64, _int, _int, _I, _I, _D, _D, _i64, _int, _int, _D, _D, _I, _int]
    lib.oracle_lu_batch.restype = None
    lib.oracle_adjoint_batch.argtypes = [_i64, _int, _int, _I, _I, _D, _D, _i64, _int, _D, _D, _dbl, _int, _int,
                                         _int, _int, _D, _D, _I, _D, _I, _int]
    lib.oracle_adjoint_batch.restype = None
    lib.oracle_mixed_batch.argtypes = [_i64, _int, _int, _I, _I, _D, _D, _i64, _int, _D, _vp, _dbl, _int, _dbl,
                                       _int, _int, _D, _I, _I, _D, _I, _int]
    lib.oracle_mixed_batch.restype = None
    lib.oracle_assemble.argtypes = [_i64, _int, _int, _I, _I, _D, _i64, _I, _I, _D, _vp, _vp]
    lib.oracle_assemble.restype = _int
    _F = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
    lib.oracle_solve_batch_f.argtypes = [_i64, _int, _int, _I, _I, _F, _F, _dbl, _int, _int, _int, _int, _F, _I, _D,
                                         _I]
    lib.oracle_solve_batch_f.restype = None
    lib.oracle_form_a.argtypes = [_int, _I, _I, _D, _dbl, _D]
    lib.oracle_form_a.restype = None
    lib.oracle_lu_solve.argtypes = [_int, _D, _D]
    lib.oracle_lu_solve.restype = _int
    lib.oracle_max_threads.argtypes = []
    lib.oracle_max_threads.restype = _int
    _lib = lib
    return lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def _prep(row_ptr, col_idx, values, gamma, b=None):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    n = rp.shape[0] - 1
    nnz = ci.shape[0]
    vals = np.ascontiguousarray(values, dtype=np.float64).reshape(-1, nnz)
    ncells = vals.shape[0]
    g = np.ascontiguousarray(np.atleast_1d(np.asarray(gamma, dtype=np.float64)))
    gstride = 0 if g.shape[0] == 1 and ncells != 1 else 1
    if gstride == 1 and g.shape[0] != ncells:
        raise ValueError("gamma must have 1 or ncells entries")
    out = [rp, ci, n, nnz, vals, ncells, g, gstride]
    if b is not None:
        bb = np.ascontiguousarray(b, dtype=np.float64).reshape(ncells, n)
        out.append(bb)
    return out


def _x0_arg(x0, C, n):
    if x0 is None:
        return None, None
    a = np.ascontiguousarray(x0, dtype=np.float64).reshape(C, n)
    return a, a.ctypes.data


PRECOND_NONE, PRECOND_JACOBI, PRECOND_ILU0 = 0, 1, 2


def solve_batch(row_ptr, col_idx, values, gamma, b, rtol=1e-10, maxit=200, precond=0, kind=J_GAMMA,
                residual_replacement=1, breakdown_restarts=1, nthreads=0, x0=None, ilu_sweeps=3):
    """precond 0 none, 1 Jacobi, 2 ILU(0) applied with ilu_sweeps Jacobi sweeps per triangle (0 = exact)."""
    rp, ci, n, nnz, vals, C, g, gs, bb = _prep(row_ptr, col_idx, values, gamma, b)
    x = np.zeros((C, n))
    iters = np.zeros(C, dtype=np.int32)
    resid = np.zeros(C)
    status = np.zeros(C, dtype=np.int32)
    x0a, x0p = _x0_arg(x0, C, n)
    _load().oracle_solve_batch(C, n, nnz, rp, ci, vals, g, gs, kind, bb, x0p, float(rtol), int(maxit), int(precond),
                               int(ilu_sweeps), int(residual_replacement), int(breakdown_restarts), x, iters, resid,
                               status, int(nthreads))
    return x, iters, resid, status


def solve_batch_f(row_ptr, col_idx, A32, b32, rtol=1e-6, maxit=200, precond=0, residual_replacement=1,
                  breakdown_restarts=1):
    """The BiCGStab of solve_batch carried out entirely in FP32 (the mixed form's inner solver), on FP32 matrices
    [ncells, nnz] (values of A) and right-hand sides, from x0 = 0.  Returns x (float32), iters, resid, status."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    n, nnz = rp.shape[0] - 1, ci.shape[0]
    A = np.ascontiguousarray(A32, dtype=np.float32).reshape(-1, nnz)
    C = A.shape[0]
    bb = np.ascontiguousarray(b32, dtype=np.float32).reshape(C, n)
    x = np.zeros((C, n), dtype=np.float32)
    iters = np.zeros(C, dtype=np.int32)
    resid = np.zeros(C)
    status = np.zeros(C, dtype=np.int32)
    _load().oracle_solve_batch_f(C, n, nnz, rp, ci, A, bb, float(rtol), int(maxit), int(precond),
                                 int(residual_replacement), int(breakdown_restarts), x, iters, resid, status)
    return x, iters, resid, status


def ilu0(row_ptr, col_idx, A):
    """ILU(0) factors (L strictly lower with unit diagonal implied, U upper) of one matrix A [nnz] on its
    pattern; raises if a row has no diagonal entry."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    Av = np.ascontiguousarray(A, dtype=np.float64)
    F = np.zeros_like(Av)
    rc = _load().oracle_ilu0(rp.shape[0] - 1, rp, ci, Av, F)
    if rc:
        raise ValueError(f"row {rc - 1} has no diagonal entry")
    return F


def ilu_apply(row_ptr, col_idx, F, p, sweeps=3):
    """(L U)^-1 p with ILU(0) factors F: exact substitution (sweeps = 0) or `sweeps` Jacobi sweeps per triangle."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    out = np.zeros(rp.shape[0] - 1)
    _load().oracle_ilu_apply(rp.shape[0] - 1, rp, ci, np.ascontiguousarray(F, dtype=np.float64), int(sweeps),
                             np.ascontiguousarray(p, dtype=np.float64), out)
    return out


def block_pattern(row_ptr, col_idx, copies):
    """CSR pattern of the block-diagonal matrix of `copies` matrices with one pattern."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    ci = np.asarray(col_idx, dtype=np.int64)
    n, nnz = rp.size - 1, ci.size
    rpg = np.concatenate([rp[:-1] + k * nnz for k in range(copies)] + [[copies * nnz]])
    cig = np.concatenate([ci + k * n for k in range(copies)])
    return rpg.astype(np.int32), cig.astype(np.int32)


def solve_groups(row_ptr, col_idx, values, gamma, b, group, rtol=1e-10, maxit=200, precond=0, kind=J_GAMMA,
                 residual_replacement=1, breakdown_restarts=1, nthreads=0):
    """Block-cells (N), Section 3: each run of `group` consecutive cells (the last run may be shorter) is one
    system, the block-diagonal matrix of its cells, solved by the same BiCGStab (solve_batch on the assembled
    system), so the cells of a run share every inner product, scalar and the stopping test.

    Per cell: x; the run's iteration count; the cell's own true relative residual ||b_c - A_c x_c|| / ||b_c||
    (0 when b_c = 0); status = the run's BREAKDOWN or NONFINITE, else CONVERGED if the cell's own residual is
    <= rtol, else MAXIT."""
    rp, ci, n, nnz, vals, C, g, gs, bb = _prep(row_ptr, col_idx, values, gamma, b)
    if group < 1:
        raise ValueError("group must be >= 1")
    if kind == J_GAMMA:
        A = np.stack([form_a(rp, ci, vals[c], g[c * gs]) for c in range(C)]) if C else vals.copy()
    else:
        A = vals
    x = np.zeros((C, n))
    iters = np.zeros(C, dtype=np.int32)
    run_status = np.zeros(C, dtype=np.int32)
    full = C // group
    for c0, runs, size in ((0, full, group), (full * group, 1 if C % group else 0, C % group)):
        if runs == 0:
            continue
        rpg, cig = block_pattern(rp, ci, size)
        m = runs * size
        xg, itg, _, stg = solve_batch(rpg, cig, A[c0:c0 + m].reshape(runs, size * nnz), [0.0],
                                      bb[c0:c0 + m].reshape(runs, size * n), rtol, maxit, precond, A_DIRECT,
                                      residual_replacement, breakdown_restarts, nthreads)
        x[c0:c0 + m] = xg.reshape(m, n)
        iters[c0:c0 + m] = np.repeat(itg, size)
        run_status[c0:c0 + m] = np.repeat(stg, size)
    ax = np.zeros((C, n))
    for i in range(n):
        ks = slice(rp[i], rp[i + 1])
        ax[:, i] = np.sum(A[:, ks] * x[:, ci[ks]], axis=1)
    bnorm = np.linalg.norm(bb, axis=1)
    rnorm = np.linalg.norm(bb - ax, axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        resid = np.where(bnorm > 0, rnorm / np.where(bnorm > 0, bnorm, 1.0), 0.0)
    status = np.where((run_status == 2) | (run_status == 3), run_status,
                      np.where(resid <= rtol, 0, 1)).astype(np.int32)
    return x, iters, resid, status


def lu_batch(row_ptr, col_idx, values, gamma, b, kind=J_GAMMA, transpose=False, nthreads=0):
    rp, ci, n, nnz, vals, C, g, gs, bb = _prep(row_ptr, col_idx, values, gamma, b)
    x = np.zeros((C, n))
    info = np.zeros(C, dtype=np.int32)
    _load().oracle_lu_batch(C, n, nnz, rp, ci, vals, g, gs, kind, int(bool(transpose)), bb, x, info,
                            int(nthreads))
    return x, info


def adjoint_batch(row_ptr, col_idx, values, gamma, x, g, rtol=1e-10, maxit=200, precond=0, kind=J_GAMMA,
                  residual_replacement=1, breakdown_restarts=1, nthreads=0):
    rp, ci, n, nnz, vals, C, gm, gs, gg = _prep(row_ptr, col_idx, values, gamma, g)
    xx = np.ascontiguousarray(x, dtype=np.float64).reshape(C, n)
    grad_b = np.zeros((C, n))
    grad_A = np.zeros((C, nnz))
    iters = np.zeros(C, dtype=np.int32)
    resid = np.zeros(C)
    status = np.zeros(C, dtype=np.int32)
    _load().oracle_adjoint_batch(C, n, nnz, rp, ci, vals, gm, gs, kind, xx, gg, float(rtol), int(maxit),
                                 int(precond), int(residual_replacement), int(breakdown_restarts), grad_b,
                                 grad_A, iters, resid, status, int(nthreads))
    return grad_b, grad_A, iters, resid, status


def mixed_batch(row_ptr, col_idx, values, gamma, b, rtol=1e-10, maxit=200, inner_rtol=1e-4, max_refine=10,
                kind=J_GAMMA, nthreads=0, budget="inner", x0=None):
    """budget "inner": maxit bounds each inner solve; "cell": the cell's inner iterations over all inner solves."""
    rp, ci, n, nnz, vals, C, g, gs, bb = _prep(row_ptr, col_idx, values, gamma, b)
    x = np.zeros((C, n))
    iters = np.zeros(C, dtype=np.int32)
    refin = np.zeros(C, dtype=np.int32)
    resid = np.zeros(C)
    status = np.zeros(C, dtype=np.int32)
    if budget not in ("inner", "cell"):
        raise ValueError("budget must be 'inner' or 'cell'")
    x0a, x0p = _x0_arg(x0, C, n)
    _load().oracle_mixed_batch(C, n, nnz, rp, ci, vals, g, gs, kind, bb, x0p, float(rtol), int(maxit),
                               float(inner_rtol), int(max_refine), int(budget == "cell"), x, iters, refin, resid,
                               status, int(nthreads))
    return x, iters, refin, resid, status


def assemble(reactants, products, k, row_ptr, col_idx, y):
    """Mass-action rates f [C, n] and Jacobian J [C, nnz] on the pattern for concentrations y [C, n].

    reactants, products: [R, 2] species indices (-1 = none); k: [R] rate constants shared by every cell, or
    [C, R] per cell."""
    reac = np.ascontiguousarray(np.asarray(reactants).reshape(-1, 2), dtype=np.int32)
    prod = np.ascontiguousarray(np.asarray(products).reshape(-1, 2), dtype=np.int32)
    R = reac.shape[0]
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    n, nnz = rp.shape[0] - 1, ci.shape[0]
    yy = np.ascontiguousarray(np.atleast_2d(y), dtype=np.float64)
    C = yy.shape[0]
    kk = np.ascontiguousarray(k, dtype=np.float64)
    ks = 0 if kk.ndim == 1 else R
    if kk.size != (R if ks == 0 else C * R):
        raise ValueError("k must have shape [R] or [C, R]")
    f = np.zeros((C, n))
    J = np.zeros((C, nnz))
    rc = _load().oracle_assemble(C, n, R, reac, prod, kk.ravel(), ks, rp, ci, yy, f.ctypes.data, J.ctypes.data)
    if rc:
        raise ValueError(f"reaction {rc - 1} needs an entry the pattern lacks")
    return f, J


def form_a(row_ptr, col_idx, J, gamma):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    Jv = np.ascontiguousarray(J, dtype=np.float64)
    A = np.zeros_like(Jv)
    _load().oracle_form_a(rp.shape[0] - 1, rp, ci, Jv, float(gamma), A)
    return A


def lu_solve_dense(A, b):
    """The oracle's own dense LU on one dense system (copies its inputs)."""
    a = np.array(A, dtype=np.float64, order="C", copy=True)
    x = np.array(b, dtype=np.float64, copy=True)
    info = _load().oracle_lu_solve(a.shape[0], a, x)
    return x, int(info)


def to_dense(row_ptr, col_idx, vals):
    """Scatter one cell's CSR values into an n x n array (test helper)."""
    n = len(row_ptr) - 1
    M = np.zeros((n, n))
    for i in range(n):
        for k in range(row_ptr[i], row_ptr[i + 1]):
            M[i, col_idx[k]] = vals[k]
    return M
