"""Shared checks of GPU results against the CPU oracle (imported by the GPU tests).

The bars (plan readings C6, C12 and the iteration/status agreement):

* x against the oracle's dense LU, on every converged cell checked.  With
  kappa = kappa_2(A) (SVD) and m = max(resid, true residual of x recomputed on
  the host, rho_LU) (rho_LU = the LU solution's own relative residual):
    - kappa * m <= 1e-8: ||x - x_LU|| / ||x_LU|| <= 1e-8, and component-wise
      |x - x_LU| <= 2 |A^-1| (|r| + |r_LU| + gamma_k (2 |b| + |A||x| + |A||x_LU|))
      with r, r_LU the host residuals of x and x_LU and gamma_k = (k + 4) u for
      rows of at most k entries (x - x* = A^-1 (b - A x) for either solution,
      plus the rounding of the host residuals and of A itself);
    - otherwise: ||x - x_LU|| / ||x_LU|| <= 4 kappa m.
* The reported residual is the true residual of the returned x, within the
  rounding of its evaluation.
* Mass-action conservation (1^T A = 1^T): |sum x - sum b| <= sqrt(n) ||b - A x||
  + 1e3 u sum |A||x|.
* Statuses and iteration counts against the oracle's BiCGStab: agreement at
  least that of the oracle with itself when b is perturbed by one ulp per
  entry (a rounding-level change), less one point; where the paper fixes no
  iteration count this is the bar (parity beyond it is unpinned).
"""
from __future__ import annotations

import numpy as np

import oracle

U64 = np.finfo(np.float64).eps / 2


def rows_of(rp):
    return np.repeat(np.arange(len(rp) - 1), np.diff(rp))


def dense_batch(rp, ci, vals):
    """[C, nnz] values on the pattern -> [C, n, n] dense."""
    n = len(rp) - 1
    C = vals.shape[0]
    D = np.zeros((C, n, n))
    D[:, rows_of(rp), ci] = vals
    return D


def a_values(rp, ci, values, gamma, kind=oracle.J_GAMMA):
    """A = I - gamma J on the pattern (the oracle's own formula), [C, nnz]."""
    if kind == oracle.A_DIRECT:
        return np.asarray(values, dtype=np.float64)
    gam = np.broadcast_to(np.atleast_1d(gamma), (values.shape[0],))
    out = np.empty_like(values)
    for c in range(values.shape[0]):
        out[c] = oracle.form_a(rp, ci, values[c], gam[c])
    return out


def lu_check(rp, ci, values, gamma, b, x, res, st, sample, kind=oracle.J_GAMMA, transpose=False,
             flat=1e-8, status_ok=0):
    """Check converged cells of `sample` against the oracle's dense LU (module docstring).
    Returns a dict of counts and the error distribution."""
    sample = np.asarray(sample)
    sample = sample[st[sample] == status_ok]
    out = {"checked": int(sample.size), "flat": 0, "kappa_bound": 0, "err_max_flat": 0.0, "err_p99": 0.0}
    if sample.size == 0:
        return out
    gam = np.broadcast_to(np.atleast_1d(gamma), (values.shape[0],))
    xl, info = oracle.lu_batch(rp, ci, values[sample], gam[sample], b[sample], kind=kind, transpose=transpose)
    Av = a_values(rp, ci, values[sample], gam[sample], kind)
    A = dense_batch(rp, ci, Av)
    if transpose:
        A = np.ascontiguousarray(np.transpose(A, (0, 2, 1)))
    kmax = int(np.max(np.diff(rp)))
    gk = (kmax + 4) * U64
    kappa = np.linalg.cond(A)
    Ainv = np.linalg.inv(A)
    bs, xs = b[sample], x[sample]
    absA = np.abs(A)
    bn = np.linalg.norm(bs, axis=1)
    r = bs - np.einsum("cij,cj->ci", A, xs)
    rl = bs - np.einsum("cij,cj->ci", A, xl)
    res_host = np.linalg.norm(r, axis=1) / bn
    rho_lu = np.linalg.norm(rl, axis=1) / bn
    Ax = np.einsum("cij,cj->ci", absA, np.abs(xs))
    Axl = np.einsum("cij,cj->ci", absA, np.abs(xl))
    # reported residual = true residual of the returned x (rounding of both evaluations)
    slack = 64 * 2 * U64 * np.linalg.norm(Ax, axis=1) / bn
    bad = np.nonzero(np.abs(res[sample] - res_host) > slack + 1e-3 * res_host)[0]
    assert bad.size == 0, ("reported residual", sample[bad[:5]], res[sample][bad[:5]], res_host[bad[:5]])
    m = np.maximum(np.maximum(res[sample], res_host), rho_lu)
    err = np.linalg.norm(xs - xl, axis=1) / np.linalg.norm(xl, axis=1)
    flat_cells = kappa * m <= flat
    # norm-wise
    lim = np.where(flat_cells, flat, 4 * kappa * m)
    bad = np.nonzero(err > lim)[0]
    assert bad.size == 0, ("x vs LU", sample[bad[:5]], err[bad[:5]], lim[bad[:5]], kappa[bad[:5]], m[bad[:5]])
    # component-wise on the cells the flat bound covers
    if flat_cells.any():
        f = flat_cells
        rhs = np.abs(r[f]) + np.abs(rl[f]) + gk * (2 * np.abs(bs[f]) + Ax[f] + Axl[f])
        cbound = 2 * np.einsum("cij,cj->ci", np.abs(Ainv[f]), rhs)
        diff = np.abs(xs[f] - xl[f])
        badc = np.argwhere(diff > cbound)
        assert badc.size == 0, ("component-wise", sample[f][badc[:5, 0]], diff[tuple(badc[:5].T)],
                                cbound[tuple(badc[:5].T)])
    out.update(flat=int(flat_cells.sum()), kappa_bound=int((~flat_cells).sum()),
               err_max_flat=float(err[flat_cells].max()) if flat_cells.any() else 0.0,
               err_p99=float(np.percentile(err, 99)), err_max=float(err.max()))
    return out


def conservation_check(rp, ci, values, gamma, b, x, st, n, chunk=20000):
    """1^T A = 1^T for the mass-action generator: sum x - sum b = -sum(b - A x)."""
    rows = rows_of(rp)
    diag = (rows == ci).astype(np.float64)
    C = values.shape[0]
    worst = 0.0
    for c0 in range(0, C, chunk):
        sl = slice(c0, min(C, c0 + chunk))
        g = np.broadcast_to(np.atleast_1d(gamma), (C,))[sl]
        A = diag[None, :] - g[:, None] * values[sl]
        xs = x[sl]
        Ax = np.zeros_like(xs)
        np.add.at(Ax.T, rows, (A * xs[:, ci]).T)
        r = b[sl] - Ax
        lhs = np.abs(xs.sum(1) - b[sl].sum(1))
        absAx = np.sum(np.abs(A) * np.abs(xs[:, ci]), axis=1)
        rhs = np.sqrt(n) * np.linalg.norm(r, axis=1) + 1e3 * U64 * absAx
        ok = st[sl] == 0
        assert np.all(lhs[ok] <= rhs[ok]), np.nonzero(ok & (lhs > rhs))[0][:5] + c0
        worst = max(worst, float(np.max(np.where(ok, lhs / np.maximum(rhs, 1e-300), 0.0))))
    return worst


def perturb_ulp(a, seed=1):
    rng = np.random.default_rng(seed)
    return a * (1 + rng.choice([-1.0, 1.0], a.shape) * 2.0 ** -52)


def perturb_ulp32(a, seed=1):
    """b perturbed at FP32 rounding level (relative 2^-24 per entry): the
    control for arithmetic carried out in FP32."""
    rng = np.random.default_rng(seed)
    return a * (1 + rng.choice([-1.0, 1.0], a.shape) * 2.0 ** -24)


def iters_close(a, b, sa, sb):
    both = (sa == 0) & (sb == 0)
    if not both.any():
        return 1.0
    return float(np.mean(np.abs(a[both] - b[both]) <= np.maximum(3, 0.15 * b[both])))
