/* CPU oracle for the batched linear systems (I - gamma*J) x = b.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * HIP library is checked against; only tests, the smoke check and the
 * benchmark's CPU-baseline leg load it.  It shares no code, header or table
 * with the HIP library.  Build: gcc -O3 -ffp-contract=off -fopenmp -shared.
 *
 * What it computes (one independent system per grid cell, Sections 2.2 and
 * 3.1: every cell has its own concentrations and Jacobian values on one shared
 * sparsity pattern, and the BDF/Newton integrator needs one linear solve per
 * step):
 *   oracle_form_a      A = I - gamma*J on the pattern (the BDF Newton matrix)
 *   oracle_solve_batch BiCGStab per cell (bicgstab_body.h), FP64
 *   oracle_lu_batch    dense LU with partial pivoting per cell (ground truth)
 *   oracle_adjoint_batch  lambda = A^-T g by BiCGStab on A^T, and the pattern
 *                      gradient dL/dA_ij = -lambda_i x_j
 *   oracle_mixed_batch FP32 inner BiCGStab + FP64 residual and refinement
 *   oracle_assemble    mass-action rates f and Jacobian J of every cell (the
 *                      inputs the linear solve needs, Section 2.2)
 * Readings of the paper taken here are listed in bicgstab_body.h and above
 * each function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_CONVERGED 0
#define OR_MAXIT 1
#define OR_BREAKDOWN 2
#define OR_NONFINITE 3

#define REAL double
#define SUFFIX d
#include "bicgstab_body.h"
#undef REAL
#undef SUFFIX

#define REAL float
#define SUFFIX f
#include "bicgstab_body.h"
#undef REAL
#undef SUFFIX

static void set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* A_k = delta_k - gamma * J_k, delta_k = 1 on diagonal positions, else 0.
 * (Newton matrix of the BDF step, Section 2.2; gamma = h * beta_0 of the
 * integrator, here given per cell.) */
void oracle_form_a(int n, const int* rp, const int* ci, const double* J, double gamma, double* A) {
  for (int i = 0; i < n; ++i)
    for (int k = rp[i]; k < rp[i + 1]; ++k) A[k] = (ci[k] == i ? 1.0 : 0.0) - gamma * J[k];
}

/* A of cell c: kind 0 = J mode (values are J, A = I - gamma*J), kind 1 = values are A. */
static void cell_matrix(int n, int nnz, const int* rp, const int* ci, const double* values,
                        const double* gamma, int64_t gamma_stride, int kind, int64_t c, double* A) {
  const double* v = values + c * (int64_t)nnz;
  if (kind == 1) {
    memcpy(A, v, sizeof(double) * (size_t)nnz);
  } else {
    oracle_form_a(n, rp, ci, v, gamma[c * gamma_stride], A);
  }
}

/* FP64 BiCGStab over a batch of cells (OpenMP over cells, static schedule).
 * x0: initial guesses [ncells, n], or NULL for zero. */
void oracle_solve_batch(int64_t ncells, int n, int nnz, const int* rp, const int* ci, const double* values,
                        const double* gamma, int64_t gamma_stride, int kind, const double* b, const double* x0,
                        double rtol, int maxit, int precond, int ilu_sweeps, int rr, int brs, double* x,
                        int32_t* iters, double* resid, int32_t* status, int nthreads) {
  set_threads(nthreads);
#pragma omp parallel
  {
    double* A = (double*)malloc(sizeof(double) * (size_t)nnz);
    double* w = (double*)malloc(sizeof(double) * 10 * (size_t)n);
#pragma omp for schedule(static)
    for (int64_t c = 0; c < ncells; ++c) {
      cell_matrix(n, nnz, rp, ci, values, gamma, gamma_stride, kind, c, A);
      int st = 0;
      iters[c] = bicgstab_d(n, rp, ci, A, b + c * n, x0 ? x0 + c * n : NULL, rtol, maxit, precond, ilu_sweeps, rr,
                            brs, x + c * n, &resid[c], &st, w);
      status[c] = st;
    }
    free(A);
    free(w);
  }
}

/* The same BiCGStab entirely in FP32 (the inner solver of the mixed form) on
 * FP32 matrices A [ncells, nnz] (A_DIRECT) and right-hand sides, x0 = 0.
 * Exposed so that the FP32 solver can be pinned on its own. */
void oracle_solve_batch_f(int64_t ncells, int n, int nnz, const int* rp, const int* ci, const float* A,
                          const float* b, double rtol, int maxit, int precond, int rr, int brs, float* x,
                          int32_t* iters, double* resid, int32_t* status) {
  float* w = (float*)malloc(sizeof(float) * 10 * (size_t)(n > 0 ? n : 1));
  for (int64_t c = 0; c < ncells; ++c) {
    int st = 0;
    iters[c] = bicgstab_f(n, rp, ci, A + c * (int64_t)nnz, b + c * n, NULL, rtol, maxit, precond, 0, rr, brs,
                          x + c * n, &resid[c], &st, w);
    status[c] = st;
  }
  free(w);
}

/* ILU(0) factors of one matrix on its pattern (see ilu0_d): F [nnz]; returns
 * 0 or i + 1 if row i has no diagonal entry. */
int oracle_ilu0(int n, const int* rp, const int* ci, const double* A, double* F) {
  int* diag = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  int rc = ilu0_d(n, rp, ci, A, F, diag);
  free(diag);
  return rc;
}

/* out = (L U)^-1 p with ILU(0) factors F, sweeps as in ilu_apply_d. */
void oracle_ilu_apply(int n, const int* rp, const int* ci, const double* F, int sweeps, const double* p,
                      double* out) {
  int* diag = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  double* t = (double*)malloc(sizeof(double) * 2 * (size_t)(n > 0 ? n : 1));
  for (int i = 0; i < n; ++i) {
    diag[i] = -1;
    for (int k = rp[i]; k < rp[i + 1]; ++k)
      if (ci[k] == i) diag[i] = k;
  }
  ilu_apply_d(n, rp, ci, F, diag, sweeps, p, out, t);
  free(diag);
  free(t);
}

/* Dense LU with partial pivoting (Doolittle; pivot = largest |a|, lowest row
 * index on ties), then forward and back substitution.  a is n*n row-major
 * and is overwritten; bx holds b on entry and x on return.  Returns 0, or
 * k+1 if the k-th pivot is exactly zero. */
int oracle_lu_solve(int n, double* a, double* bx) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = fabs(a[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double m = fabs(a[(size_t)i * n + k]);
      if (m > best) { best = m; p = i; }
    }
    if (best == 0.0) return k + 1;
    if (p != k) {
      for (int j = 0; j < n; ++j) {
        double tmp = a[(size_t)k * n + j];
        a[(size_t)k * n + j] = a[(size_t)p * n + j];
        a[(size_t)p * n + j] = tmp;
      }
      double tb = bx[k]; bx[k] = bx[p]; bx[p] = tb;
    }
    double piv = a[(size_t)k * n + k];
    for (int i = k + 1; i < n; ++i) {
      double l = a[(size_t)i * n + k] / piv;
      a[(size_t)i * n + k] = l;
      for (int j = k + 1; j < n; ++j) a[(size_t)i * n + j] -= l * a[(size_t)k * n + j];
      bx[i] -= l * bx[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = bx[i];
    for (int j = i + 1; j < n; ++j) s -= a[(size_t)i * n + j] * bx[j];
    bx[i] = s / a[(size_t)i * n + i];
  }
  return 0;
}

/* Dense LU solve per cell of A x = b (transpose = 0) or A^T x = b (transpose = 1).
 * info[c] = oracle_lu_solve's return. */
void oracle_lu_batch(int64_t ncells, int n, int nnz, const int* rp, const int* ci, const double* values,
                     const double* gamma, int64_t gamma_stride, int kind, int transpose, const double* b,
                     double* x, int32_t* info, int nthreads) {
  set_threads(nthreads);
#pragma omp parallel
  {
    double* A = (double*)malloc(sizeof(double) * (size_t)nnz);
    double* D = (double*)malloc(sizeof(double) * (size_t)n * n);
#pragma omp for schedule(static)
    for (int64_t c = 0; c < ncells; ++c) {
      cell_matrix(n, nnz, rp, ci, values, gamma, gamma_stride, kind, c, A);
      memset(D, 0, sizeof(double) * (size_t)n * n);
      for (int i = 0; i < n; ++i)
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
          if (transpose) D[(size_t)ci[k] * n + i] = A[k];
          else D[(size_t)i * n + ci[k]] = A[k];
        }
      for (int i = 0; i < n; ++i) x[c * n + i] = b[c * n + i];
      info[c] = oracle_lu_solve(n, D, x + c * n);
    }
    free(A);
    free(D);
  }
}

/* CSR of A^T from CSR of A: trp/tci describe the transposed pattern and
 * perm[q] is the position in A of the q-th entry of A^T. */
void oracle_transpose_pattern(int n, const int* rp, const int* ci, int* trp, int* tci, int* perm) {
  int nnz = rp[n];
  for (int j = 0; j <= n; ++j) trp[j] = 0;
  for (int k = 0; k < nnz; ++k) trp[ci[k] + 1]++;
  for (int j = 0; j < n; ++j) trp[j + 1] += trp[j];
  int* fill = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  for (int j = 0; j < n; ++j) fill[j] = trp[j];
  for (int i = 0; i < n; ++i)
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      int q = fill[ci[k]]++;
      tci[q] = i;
      perm[q] = k;
    }
  free(fill);
}

/* Adjoint of the solve with loss L(x): given x (the forward solution) and
 * g = dL/dx, solve A^T lambda = g with the same BiCGStab, then
 *   dL/db = lambda,  dL/dA_k = -lambda_i * x_j for pattern entry k = (i, j).
 * (Differentiating A x = b: dx = A^-1 (db - dA x), so dL = lambda^T db -
 * lambda^T dA x.) */
void oracle_adjoint_batch(int64_t ncells, int n, int nnz, const int* rp, const int* ci, const double* values,
                          const double* gamma, int64_t gamma_stride, int kind, const double* x, const double* g,
                          double rtol, int maxit, int precond, int rr, int brs, double* grad_b, double* grad_A,
                          int32_t* iters, double* resid, int32_t* status, int nthreads) {
  int* trp = (int*)malloc(sizeof(int) * (size_t)(n + 1));
  int* tci = (int*)malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
  int* perm = (int*)malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
  oracle_transpose_pattern(n, rp, ci, trp, tci, perm);
  set_threads(nthreads);
#pragma omp parallel
  {
    double* A = (double*)malloc(sizeof(double) * (size_t)nnz);
    double* AT = (double*)malloc(sizeof(double) * (size_t)nnz);
    double* w = (double*)malloc(sizeof(double) * 10 * (size_t)n);
#pragma omp for schedule(static)
    for (int64_t c = 0; c < ncells; ++c) {
      cell_matrix(n, nnz, rp, ci, values, gamma, gamma_stride, kind, c, A);
      for (int q = 0; q < nnz; ++q) AT[q] = A[perm[q]];
      int st = 0;
      double* lam = grad_b + c * n;
      iters[c] = bicgstab_d(n, trp, tci, AT, g + c * n, NULL, rtol, maxit, precond, 0, rr, brs, lam, &resid[c],
                            &st, w);
      status[c] = st;
      const double* xc = x + c * n;
      for (int i = 0; i < n; ++i)
        for (int k = rp[i]; k < rp[i + 1]; ++k) grad_A[c * nnz + k] = -lam[i] * xc[ci[k]];
    }
    free(A);
    free(AT);
    free(w);
  }
  free(trp);
  free(tci);
  free(perm);
}

/* Mixed precision: FP32 inner BiCGStab inside FP64 iterative refinement.
 *   D = diag(A) (FP64); Ahat = A D^-1 (FP64 division, then rounded to float);
 *   x = x0 (or 0), r = b - A x;
 *   repeat up to max_refine times while ||r||/||b|| > rtol (and, with
 *   budget_cell, while fewer than maxit inner iterations were spent: maxit is
 *   then the cell's iteration budget over all inner solves):
 *     rhat32 = float(r / ||r||);
 *     solve Ahat d = rhat32 in FP32 to inner_rtol (no residual replacement)
 *     within maxit iterations (budget_cell: the cell's remaining budget);
 *     x_new = x + ||r|| * D^-1 * d (FP64); r_new = b - A x_new (FP64);
 *     if ||r_new|| >= ||r||: stop (refinement stagnates; x is kept).
 * iters = sum of inner iterations, refinements = inner solves performed.
 * Status: CONVERGED if the final FP64 relative residual <= rtol, NONFINITE on
 * non-finite values, otherwise MAXIT. */
void oracle_mixed_batch(int64_t ncells, int n, int nnz, const int* rp, const int* ci, const double* values,
                        const double* gamma, int64_t gamma_stride, int kind, const double* b, const double* x0,
                        double rtol, int maxit, double inner_rtol, int max_refine, int budget_cell, double* x,
                        int32_t* iters, int32_t* refinements, double* resid, int32_t* status, int nthreads) {
  set_threads(nthreads);
#pragma omp parallel
  {
    double* A = (double*)malloc(sizeof(double) * (size_t)nnz);
    float* A32 = (float*)malloc(sizeof(float) * (size_t)nnz);
    double* dg = (double*)malloc(sizeof(double) * (size_t)n);
    double* r = (double*)malloc(sizeof(double) * (size_t)n);
    double* xn = (double*)malloc(sizeof(double) * (size_t)n);
    double* rn_v = (double*)malloc(sizeof(double) * (size_t)n);
    float* r32 = (float*)malloc(sizeof(float) * (size_t)n);
    float* d32 = (float*)malloc(sizeof(float) * (size_t)n);
    float* w32 = (float*)malloc(sizeof(float) * 10 * (size_t)n);
#pragma omp for schedule(static)
    for (int64_t c = 0; c < ncells; ++c) {
      cell_matrix(n, nnz, rp, ci, values, gamma, gamma_stride, kind, c, A);
      const double* bc = b + c * n;
      double* xc = x + c * n;
      int tot = 0, nref = 0, st = OR_MAXIT;
      for (int i = 0; i < n; ++i) xc[i] = 0.0;
      double bn = 0.0;
      for (int i = 0; i < n; ++i) bn += bc[i] * bc[i];
      bn = sqrt(bn);
      double res;
      if (!isfinite(bn)) {
        res = NAN;
        st = OR_NONFINITE;
      } else if (bn == 0.0) {
        res = 0.0;
        st = OR_CONVERGED;
      } else {
        for (int i = 0; i < n; ++i) {
          double d = 0.0;
          for (int k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] == i) d = A[k];
          dg[i] = d;
        }
        for (int i = 0; i < n; ++i)
          for (int k = rp[i]; k < rp[i + 1]; ++k) A32[k] = (float)(A[k] / dg[ci[k]]);
        double rn = bn;
        if (x0) {
          for (int i = 0; i < n; ++i) xc[i] = x0[c * n + i];
          for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int k = rp[i]; k < rp[i + 1]; ++k) acc += A[k] * xc[ci[k]];
            r[i] = bc[i] - acc;
          }
          rn = 0.0;
          for (int i = 0; i < n; ++i) rn += r[i] * r[i];
          rn = sqrt(rn);
        } else {
          for (int i = 0; i < n; ++i) r[i] = bc[i];
        }
        while (1) {
          if (!isfinite(rn)) { st = OR_NONFINITE; break; }
          if (rn / bn <= rtol) { st = OR_CONVERGED; break; }
          if (nref >= max_refine || (budget_cell && tot >= maxit)) { st = OR_MAXIT; break; }
          for (int i = 0; i < n; ++i) r32[i] = (float)(r[i] / rn);
          double ires;
          int ist;
          tot += bicgstab_f(n, rp, ci, A32, r32, NULL, inner_rtol, budget_cell ? maxit - tot : maxit, 0, 0, 0, 1,
                            d32, &ires, &ist, w32);
          ++nref;
          if (ist == OR_NONFINITE) { st = OR_NONFINITE; break; }
          for (int i = 0; i < n; ++i) xn[i] = xc[i] + rn * ((double)d32[i] / dg[i]);
          for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int k = rp[i]; k < rp[i + 1]; ++k) acc += A[k] * xn[ci[k]];
            rn_v[i] = bc[i] - acc;
          }
          double rnn = 0.0;
          for (int i = 0; i < n; ++i) rnn += rn_v[i] * rn_v[i];
          rnn = sqrt(rnn);
          if (!(rnn < rn)) { st = isfinite(rnn) ? OR_MAXIT : OR_NONFINITE; break; }
          for (int i = 0; i < n; ++i) { xc[i] = xn[i]; r[i] = rn_v[i]; }
          rn = rnn;
        }
        res = rn / bn;
        if (st == OR_NONFINITE) res = NAN;
      }
      iters[c] = tot;
      refinements[c] = nref;
      resid[c] = res;
      status[c] = st;
    }
    free(A); free(A32); free(dg); free(r); free(xn); free(rn_v); free(r32); free(d32); free(w32);
  }
}

/* Mass-action rates and their Jacobian, per cell (the chemistry of Section
 * 2.2: the rate of change of each species is a sum over reactions, and the
 * BDF step needs the Jacobian of that rate function).  Reaction r consumes
 * reactants reac[2r] and reac[2r+1] (-1 = none) and makes products
 * prod[2r], prod[2r+1] (-1 = none) at the mass-action rate
 *   w_r = k_r y_a            (one reactant a)
 *   w_r = (k_r y_a) y_b      (two reactants a, b; a == b allowed)
 * with k_r = k[c * k_stride + r] (k_stride 0: one set for every cell).
 * f_i = sum_r S_ir w_r, S_ir = (times i is a product) - (times i is a
 * reactant); J_ij = d f_i / d y_j = sum_r S_ir d w_r / d y_j with
 *   d w / d y_a = k_r               (one reactant)
 *   d w / d y_a = k_r y_b, d w / d y_b = k_r y_a   (a != b)
 *   d w / d y_a = 2 (k_r y_a)       (a == b).
 * Reactions are taken in order and, within one, the species in the order
 * reactants then products, each species once; J is written on the CSR
 * pattern (rp, ci).  f or J may be NULL.  Returns 0, or 1 + r if reaction r
 * needs an entry the pattern lacks (nothing is then guaranteed). */
int oracle_assemble(int64_t ncells, int n, int R, const int* reac, const int* prod, const double* k,
                    int64_t k_stride, const int* rp, const int* ci, const double* y, double* f, double* J) {
  int nnz = rp[n];
  for (int64_t c = 0; c < ncells; ++c) {
    const double* yc = y + c * n;
    if (f)
      for (int i = 0; i < n; ++i) f[c * n + i] = 0.0;
    if (J)
      for (int q = 0; q < nnz; ++q) J[c * nnz + q] = 0.0;
    for (int r = 0; r < R; ++r) {
      double kr = k[c * k_stride + r];
      int a = reac[2 * r], b = reac[2 * r + 1];
      /* species of the reaction with their net stoichiometry */
      int sp[4], ns = 0;
      double st[4];
      int all[4] = {reac[2 * r], reac[2 * r + 1], prod[2 * r], prod[2 * r + 1]};
      for (int q = 0; q < 4; ++q) {
        if (all[q] < 0) continue;
        double d = q < 2 ? -1.0 : 1.0;
        int found = -1;
        for (int u = 0; u < ns; ++u)
          if (sp[u] == all[q]) found = u;
        if (found < 0) {
          sp[ns] = all[q];
          st[ns] = d;
          ++ns;
        } else {
          st[found] += d;
        }
      }
      double w = kr * yc[a];
      if (b >= 0) w = w * yc[b];
      /* derivative of w by each reactant */
      int dj[2];
      double dw[2];
      int nd = 0;
      if (b < 0) {
        dj[0] = a;
        dw[0] = kr;
        nd = 1;
      } else if (a == b) {
        dj[0] = a;
        dw[0] = 2.0 * (kr * yc[a]);
        nd = 1;
      } else {
        dj[0] = a;
        dw[0] = kr * yc[b];
        dj[1] = b;
        dw[1] = kr * yc[a];
        nd = 2;
      }
      for (int u = 0; u < ns; ++u) {
        int i = sp[u];
        if (f) f[c * n + i] = f[c * n + i] + st[u] * w;
        if (!J) continue;
        for (int v = 0; v < nd; ++v) {
          int pos = -1;
          for (int q = rp[i]; q < rp[i + 1]; ++q)
            if (ci[q] == dj[v]) pos = q;
          if (pos < 0) return 1 + r;
          J[c * nnz + pos] = J[c * nnz + pos] + st[u] * dw[v];
        }
      }
    }
  }
  return 0;
}
