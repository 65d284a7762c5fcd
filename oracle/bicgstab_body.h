/* One BiCGStab solve of A x = b on a CSR matrix, written once and compiled for
 * two element types by oracle.c (REAL = double for the FP64 oracle, REAL =
 * float for the inner solve of the mixed-precision emulation).
 *
 * TEST INFRASTRUCTURE: part of the CPU oracle; nothing on the product path
 * uses it.
 *
 * Method: BiCGStab of van der Vorst (1992), as given in the BiCGSTAB template
 * of Barrett et al., "Templates for the Solution of Linear Systems" (SIAM
 * 1994), with optional right preconditioning: Jacobi, M = diag(A), or
 * ILU(0), M = L U with the incomplete factors on A's own pattern (Saad,
 * Iterative Methods for Sparse Linear Systems, 2nd ed., Algorithm 10.4; the
 * paper names a preconditioner as the most promising next optimisation,
 * Section 5.2).  The paper
 * names its linear solver only as the BSC "Biconjugate Gradient" GPU solver
 * (Section 3.1) and prints no algorithm, so the published BiCGStab is
 * followed.  Readings taken where the paper is silent:
 *   - initial guess x0 = 0 unless the caller gives one, shadow residual
 *     rhat = r0 = b - A x0; a cell whose initial residual already meets
 *     rtol takes no iteration;
 *   - stop when ||s||/||b|| or ||r||/||b|| (2-norm, recurrence residual) is
 *     <= rtol, then confirm on the true residual ||b - A x||/||b||;
 *   - if the true residual misses rtol: residual replacement (r <- b - A x,
 *     restart the recurrences) while iterations remain;
 *   - breakdown = an exact zero rho, sigma, tau or omega: restart from the
 *     true residual up to `brs` times, then stop with status BREAKDOWN;
 *   - any non-finite scalar stops the cell with status NONFINITE;
 *   - the iteration count counts loop entries (a half-step exit counts 1).
 * Dot products and norms accumulate sequentially in index order.
 */

#ifndef REAL
#error "define REAL before including bicgstab_body.h"
#endif
#ifndef SUFFIX
#error "define SUFFIX before including bicgstab_body.h"
#endif

#define CAT2(a, b) a##b
#define CAT(a, b) CAT2(a, b)
#define FN(name) CAT(name, SUFFIX)

static REAL FN(dot_)(int n, const REAL* a, const REAL* b) {
  REAL s = 0;
  for (int i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

static REAL FN(nrm2_)(int n, const REAL* a) { return (REAL)sqrt((double)FN(dot_)(n, a, a)); }

/* y = A x on the CSR pattern (row order, column order within a row). */
static void FN(spmv_)(int n, const int* rp, const int* ci, const REAL* A, const REAL* xv, REAL* y) {
  for (int i = 0; i < n; ++i) {
    REAL acc = 0;
    for (int k = rp[i]; k < rp[i + 1]; ++k) acc += A[k] * xv[ci[k]];
    y[i] = acc;
  }
}

/* ILU(0) of A on its own pattern (Saad, Algorithm 10.4, the IKJ variant):
 * for each row i and each k < i with (i, k) in the pattern, in increasing k:
 * a_ik <- a_ik / a_kk, then a_ij <- a_ij - a_ik a_kj for every j > k with both
 * (i, j) and (k, j) in the pattern.  F receives L (strictly lower part, unit
 * diagonal implied) and U (diagonal and upper part) on the pattern; diag[i]
 * is the position of (i, i).  Returns 0, or i + 1 if row i has no diagonal
 * entry.  A zero pivot is not trapped: the division gives an infinity and
 * the solve reports a non-finite value. */
static int FN(ilu0_)(int n, const int* rp, const int* ci, const REAL* A, REAL* F, int* diag) {
  int nnz = rp[n];
  for (int k = 0; k < nnz; ++k) F[k] = A[k];
  for (int i = 0; i < n; ++i) {
    diag[i] = -1;
    for (int k = rp[i]; k < rp[i + 1]; ++k)
      if (ci[k] == i) diag[i] = k;
    if (diag[i] < 0) return i + 1;
  }
  for (int i = 1; i < n; ++i) {
    for (int pk = rp[i]; pk < rp[i + 1] && ci[pk] < i; ++pk) {
      int k = ci[pk];
      F[pk] = F[pk] / F[diag[k]];
      for (int pj = pk + 1; pj < rp[i + 1]; ++pj) {
        int j = ci[pj];
        for (int q = diag[k] + 1; q < rp[k + 1]; ++q)
          if (ci[q] == j) {
            F[pj] = F[pj] - F[pk] * F[q];
            break;
          }
      }
    }
  }
  return 0;
}

/* out = (L U)^-1 p with the ILU(0) factors F.  sweeps = 0: exact forward and
 * back substitution.  sweeps = s > 0: each triangular system solved by s
 * Jacobi sweeps from the diagonal solution (L y = p: y <- p, then s times
 * y <- p - L_strict y; U z = y: z <- D^-1 y, then s times
 * z <- D^-1 (y - U_strict z)), a fixed linear operator (the truncated
 * Neumann series), exact once s reaches the depth of the triangle.  t must
 * hold 2n elements. */
static void FN(ilu_apply_)(int n, const int* rp, const int* ci, const REAL* F, const int* diag, int sweeps,
                           const REAL* p, REAL* out, REAL* t) {
  REAL *y = t, *u = t + n;
  if (sweeps == 0) {
    for (int i = 0; i < n; ++i) {
      REAL acc = p[i];
      for (int k = rp[i]; k < diag[i]; ++k) acc -= F[k] * y[ci[k]];
      y[i] = acc;
    }
    for (int i = n - 1; i >= 0; --i) {
      REAL acc = y[i];
      for (int k = diag[i] + 1; k < rp[i + 1]; ++k) acc -= F[k] * out[ci[k]];
      out[i] = acc / F[diag[i]];
    }
    return;
  }
  for (int i = 0; i < n; ++i) y[i] = p[i];
  for (int sw = 0; sw < sweeps; ++sw) {
    for (int i = 0; i < n; ++i) {
      REAL acc = p[i];
      for (int k = rp[i]; k < diag[i]; ++k) acc -= F[k] * y[ci[k]];
      u[i] = acc;
    }
    for (int i = 0; i < n; ++i) y[i] = u[i];
  }
  for (int i = 0; i < n; ++i) out[i] = y[i] / F[diag[i]];
  for (int sw = 0; sw < sweeps; ++sw) {
    for (int i = 0; i < n; ++i) {
      REAL acc = y[i];
      for (int k = diag[i] + 1; k < rp[i + 1]; ++k) acc -= F[k] * out[ci[k]];
      u[i] = acc / F[diag[i]];
    }
    for (int i = 0; i < n; ++i) out[i] = u[i];
  }
}

/* Returns the iteration count.  x0 is the initial guess (NULL: zero).
 * precond: 0 none, 1 Jacobi, 2 ILU(0) applied with ilu_sweeps (0 = exact).
 * w must hold 10*n elements. */
static int FN(bicgstab_core_)(int n, const int* rp, const int* ci, const REAL* A, const REAL* b, const REAL* x0,
                              double rtol, int maxit, int precond, int ilu_sweeps, int rr, int brs, REAL* x,
                              double* resid_out, int* status_out, REAL* w, const REAL* F, const int* fdiag,
                              REAL* ft) {
  REAL *r = w, *rh = w + n, *p = w + 2 * n, *v = w + 3 * n, *s = w + 4 * n;
  REAL *t = w + 5 * n, *ph = w + 6 * n, *sh = w + 7 * n, *dinv = w + 8 * n, *rt = w + 9 * n;
  for (int i = 0; i < n; ++i) x[i] = 0;
  REAL bn = FN(nrm2_)(n, b);
  if (!isfinite((double)bn)) {
    *resid_out = NAN;
    *status_out = OR_NONFINITE;
    return 0;
  }
  if (bn == 0) {
    *resid_out = 0.0;
    *status_out = OR_CONVERGED;
    return 0;
  }
  if (precond == 1) {
    for (int i = 0; i < n; ++i) {
      REAL d = 0;
      for (int k = rp[i]; k < rp[i + 1]; ++k)
        if (ci[k] == i) d = A[k];
      dinv[i] = (REAL)1 / d;
    }
  }
#define PRECOND_APPLY(dst, src)                                                \
  do {                                                                         \
    if (precond == 2)                                                          \
      FN(ilu_apply_)(n, rp, ci, F, fdiag, ilu_sweeps, src, dst, ft);           \
    else                                                                       \
      for (int i_ = 0; i_ < n; ++i_) dst[i_] = precond ? dinv[i_] * src[i_] : src[i_]; \
  } while (0)
  /* r0 = b - A x0 */
  if (x0) {
    for (int i = 0; i < n; ++i) x[i] = x0[i];
    FN(spmv_)(n, rp, ci, A, x, rt);
    for (int i = 0; i < n; ++i) r[i] = b[i] - rt[i];
  } else {
    for (int i = 0; i < n; ++i) r[i] = b[i];
  }
  {
    double r0 = (double)FN(nrm2_)(n, r) / (double)bn;
    if (r0 <= rtol) {
      *resid_out = r0;
      *status_out = OR_CONVERGED;
      return 0;
    }
  }

  int it = 0, restarts_left = brs, ended = OR_MAXIT;
  double res = 0.0;
  for (;;) {
    /* (re)start the recurrences from the current r */
    for (int i = 0; i < n; ++i) rh[i] = r[i];
    REAL rho_prev = 1, alpha = 1, omega = 1;
    int first = 1;
    ended = OR_MAXIT;
    while (it < maxit) {
      ++it;
      REAL rho = FN(dot_)(n, rh, r);
      if (!isfinite((double)rho)) { ended = OR_NONFINITE; break; }
      if (rho == 0) { ended = OR_BREAKDOWN; break; }
      if (first) {
        for (int i = 0; i < n; ++i) p[i] = r[i];
        first = 0;
      } else {
        REAL beta = (rho / rho_prev) * (alpha / omega);
        for (int i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
      }
      PRECOND_APPLY(ph, p);
      FN(spmv_)(n, rp, ci, A, ph, v);
      REAL sigma = FN(dot_)(n, rh, v);
      if (!isfinite((double)sigma)) { ended = OR_NONFINITE; break; }
      if (sigma == 0) { ended = OR_BREAKDOWN; break; }
      alpha = rho / sigma;
      for (int i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
      REAL sn = FN(nrm2_)(n, s);
      if (!isfinite((double)sn)) { ended = OR_NONFINITE; break; }
      if ((double)sn / (double)bn <= rtol) {
        for (int i = 0; i < n; ++i) x[i] = x[i] + alpha * ph[i];
        ended = OR_CONVERGED;
        break;
      }
      PRECOND_APPLY(sh, s);
      FN(spmv_)(n, rp, ci, A, sh, t);
      REAL tau = FN(dot_)(n, t, t);
      if (!isfinite((double)tau)) { ended = OR_NONFINITE; break; }
      if (tau == 0) { ended = OR_BREAKDOWN; break; }
      omega = FN(dot_)(n, t, s) / tau;
      for (int i = 0; i < n; ++i) x[i] = x[i] + alpha * ph[i] + omega * sh[i];
      for (int i = 0; i < n; ++i) r[i] = s[i] - omega * t[i];
      REAL rn = FN(nrm2_)(n, r);
      if (!isfinite((double)rn)) { ended = OR_NONFINITE; break; }
      if ((double)rn / (double)bn <= rtol) { ended = OR_CONVERGED; break; }
      if (omega == 0) { ended = OR_BREAKDOWN; break; }
      rho_prev = rho;
    }
    /* true residual of the current iterate */
    FN(spmv_)(n, rp, ci, A, x, rt);
    for (int i = 0; i < n; ++i) rt[i] = b[i] - rt[i];
    res = (double)FN(nrm2_)(n, rt) / (double)bn;
    if (ended == OR_NONFINITE || !isfinite(res)) {
      *resid_out = res;
      *status_out = OR_NONFINITE;
      return it;
    }
    if (res <= rtol) {
      *resid_out = res;
      *status_out = OR_CONVERGED;
      return it;
    }
    if (it < maxit && ((ended == OR_CONVERGED && rr) || (ended == OR_BREAKDOWN && restarts_left > 0))) {
      if (ended == OR_BREAKDOWN) --restarts_left;
      for (int i = 0; i < n; ++i) r[i] = rt[i];
      continue;
    }
    *resid_out = res;
    *status_out = (ended == OR_BREAKDOWN) ? OR_BREAKDOWN : OR_MAXIT;
    return it;
  }
}

#undef PRECOND_APPLY

static int FN(bicgstab_)(int n, const int* rp, const int* ci, const REAL* A, const REAL* b, const REAL* x0,
                         double rtol, int maxit, int precond, int ilu_sweeps, int rr, int brs, REAL* x,
                         double* resid_out, int* status_out, REAL* w) {
  if (precond != 2)
    return FN(bicgstab_core_)(n, rp, ci, A, b, x0, rtol, maxit, precond, ilu_sweeps, rr, brs, x, resid_out,
                              status_out, w, NULL, NULL, NULL);
  REAL* F = (REAL*)malloc(sizeof(REAL) * (size_t)(rp[n] > 0 ? rp[n] : 1));
  int* fdiag = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  REAL* ft = (REAL*)malloc(sizeof(REAL) * 2 * (size_t)(n > 0 ? n : 1));
  FN(ilu0_)(n, rp, ci, A, F, fdiag); /* the pattern's diagonal is checked by the caller */
  int it = FN(bicgstab_core_)(n, rp, ci, A, b, x0, rtol, maxit, precond, ilu_sweeps, rr, brs, x, resid_out,
                              status_out, w, F, fdiag, ft);
  free(F);
  free(fdiag);
  free(ft);
  return it;
}

#undef FN
#undef CAT
#undef CAT2
