/* bcs.h -- batched Block-cells BiCGStab for (I - gamma*J) x = b on AMD gfx950.
 *
 * One small sparse linear system per grid cell.  All cells share one sparsity
 * pattern (the chemical Jacobian's, Section 2.2: CAMP stores the Jacobian
 * sparse, and in the multi-cell form each species y_ik belongs to a cell k);
 * every cell has its own values.  Each cell is solved entirely inside one
 * workgroup, with no communication between workgroups and no host round trip
 * during the solve (the Block-cells arrangement of Section 3.1, whose BCG
 * solver is realised here as BiCGStab).  The linear system is the Newton
 * matrix of the BDF integrator, which needs one linear solve per step
 * (Section 2.2).
 *
 * Conventions for every entry point:
 *   - Pattern arrays passed to bcs_plan_create are HOST pointers; they are
 *     copied, the caller keeps ownership.
 *   - Every per-cell array passed to a solve is a DEVICE pointer owned by the
 *     caller (e.g. torch tensors); the library never allocates, frees or
 *     retains them.  Layouts are row-major, cell-major: values [ncells, nnz]
 *     in the CSR order of the plan's pattern, vectors [ncells, n].
 *   - Solves are asynchronous on `stream` (a hipStream_t; NULL = the default
 *     stream).  Outputs are valid once the stream has been synchronised.
 *   - Solves allocate no memory.  Their scratch (the work queue of the
 *     persistent grid and the cells' cost order) lives in a caller-owned
 *     DEVICE `workspace` of at least bcs_workspace_bytes(plan, ncells) bytes,
 *     256-byte aligned, which the solve initialises itself on `stream` (no
 *     memset needed; any previous contents are ignored).  A plan holds no
 *     mutable state: several solves with one plan may run at the same time
 *     (different streams or host threads) provided each has its own
 *     workspace.  Solves that share a workspace race unless serialised.
 *   - Return value: BCS_OK (0), or a negative BCS_ERR_* code for argument,
 *     pattern, support or HIP runtime errors, detected synchronously before
 *     any launch; bcs_last_error() then describes it (thread-local string).
 *     Numerical outcomes are never return codes: they are per-cell in
 *     `status`.
 *   - ncells == 0 is a no-op that returns BCS_OK.
 */
#ifndef BCS_H
#define BCS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define BCS_OK 0
#define BCS_ERR_ARG (-1)         /* bad argument (null pointer, size, option value) */
#define BCS_ERR_PATTERN (-2)     /* invalid CSR pattern */
#define BCS_ERR_UNSUPPORTED (-3) /* valid but outside what the kernels handle (e.g. n too large) */
#define BCS_ERR_HIP (-4)         /* HIP runtime error (allocation, copy, launch) */

/* per-cell status */
#define BCS_CONVERGED 0 /* true relative residual ||b - A x||/||b|| <= rtol */
#define BCS_MAXIT 1     /* stopped without reaching rtol (iteration or refinement budget spent) */
#define BCS_BREAKDOWN 2 /* exact-zero rho, sigma, tau or omega after the allowed restarts */
#define BCS_NONFINITE 3 /* a non-finite value appeared (NaN/Inf in inputs or iterates) */

/* options */
#define BCS_FP64 0        /* all arithmetic in FP64 */
#define BCS_FP32_REFINE 1 /* FP32 inner BiCGStab, FP64 residual, scaling and update */
#define BCS_PRECOND_NONE 0
#define BCS_PRECOND_JACOBI 1 /* right preconditioning with M = diag(A) */
#define BCS_PRECOND_ILU0 2   /* right preconditioning with M = L U, the incomplete LU
                                factors of A on A's own pattern (ILU(0)); the paper
                                names a preconditioner as its solver's most promising
                                next optimisation (Section 5.2).  The factors are
                                computed per cell inside the solve; M^-1 is applied by
                                ilu_sweeps Jacobi sweeps per triangular factor.  FP64,
                                jit = 1, forward solves (bcs_solve_batch) only */
#define BCS_J_GAMMA 0        /* values hold J; A = I - gamma*J (pattern must hold the diagonal) */
#define BCS_A_DIRECT 1       /* values hold A itself; gamma is ignored */
#define BCS_BUDGET_INNER 0   /* FP32_REFINE: maxit bounds each inner solve */
#define BCS_BUDGET_CELL 1    /* FP32_REFINE: maxit bounds a cell's inner iterations over all inner solves */

typedef struct bcs_options {
  int32_t precision;            /* BCS_FP64 | BCS_FP32_REFINE                          */
  int32_t precond;              /* BCS_PRECOND_NONE | BCS_PRECOND_JACOBI               */
  int32_t matrix_kind;          /* BCS_J_GAMMA | BCS_A_DIRECT                          */
  int32_t lanes_per_cell;       /* 0 = choose; else 16, 32 or 64 lanes own one cell   */
  int32_t residual_replacement; /* 1: on a recurrence-only convergence, restart from
                                   the true residual while iterations remain          */
  int32_t breakdown_restarts;   /* restarts allowed after an exact breakdown          */
  double inner_rtol;            /* FP32_REFINE: inner solve tolerance (relative)      */
  int32_t max_refine;           /* FP32_REFINE: maximum number of inner solves        */
  int32_t jit;                  /* 1: compile kernels specialised to this pattern at
                                   plan creation (hipRTC; cached on disk under
                                   $BCS_JIT_CACHE or ~/.cache/bcs_jit); 0: use the
                                   precompiled generic kernels                       */
  int32_t autotune;             /* 1: with lanes_per_cell == 0, time the candidate
                                   layouts on a synthetic batch of this pattern (a
                                   spread of diagonally dominant cells) and keep the
                                   fastest; 0: choose by a cost model; see also
                                   bcs_plan_autotune for tuning on real data        */
  int32_t cell_order;           /* 1: in a BCS_J_GAMMA solve with one gamma per cell,
                                   hand the cells to the solver in a cost order:
                                   cells sorted by gamma on the device (small
                                   kernels on the solve's stream), handed out
                                   alternately from the large-gamma and the
                                   small-gamma end, so that expensive cells start
                                   early.  Applied only when the batch has more
                                   cells than the launch has cell slots (with
                                   no more, slot k solves cell k: every cell
                                   starts at once, and nothing runs before the
                                   solve kernel).
                                   Results are identical to index order.
                                   0: index order                                  */
  int32_t shared_scalars;       /* 1: Block-cells (N) of Section 3, an experiment
                                   mode: each run of 64 / lanes_per_cell consecutive
                                   cells (one wave's cells; the last run may be
                                   shorter) is solved as one system, the block-
                                   diagonal matrix of its cells, so the run shares
                                   every inner product, scalar and stopping test.
                                   Each cell reports the run's iteration count, its
                                   own true relative residual, and BCS_CONVERGED
                                   only if that residual is <= rtol (else
                                   BCS_MAXIT, or the run's BREAKDOWN / NONFINITE).
                                   Needs FP64, jit = 1 and lanes_per_cell 16, 32 or
                                   64 (1 cell per run); forward solves only, cells
                                   in index order, no initial guess.  0: every cell
                                   on its own                                      */
  int32_t refine_budget;        /* FP32_REFINE: BCS_BUDGET_INNER (each inner solve
                                   may take maxit iterations, at most max_refine
                                   inner solves) or BCS_BUDGET_CELL (maxit bounds the
                                   cell's inner iterations summed over its inner
                                   solves, as it bounds the FP64 solve's iterations
                                   summed over its restarts)                       */
  int32_t ilu_sweeps;           /* BCS_PRECOND_ILU0: Jacobi sweeps per triangular
                                   solve, 1..16 (0 = the library's default, 3): L y = q
                                   by y <- q, then ilu_sweeps times y <- q - L_s y;
                                   U z = y by z <- D^-1 y, then ilu_sweeps times
                                   z <- D^-1 (y - U_s z) (L_s, U_s the strict parts,
                                   D = diag(U)), the truncated Neumann series of each
                                   factor.  Must be 0 for other preconditioners    */
  int32_t waves_per_group;      /* waves per workgroup of the forward FP64 kernel
                                   (Section 3.2's threads per block; a workgroup's
                                   waves share only its copy of the schedule): 0 =
                                   4, which bcs_plan_autotune may change to 2 or 8
                                   when that is more than 3% faster; 1, 2, 4 or 8
                                   fix it (jit = 1, FP64, not ILU0, no
                                   shared_scalars, else BCS_ERR_UNSUPPORTED)       */
} bcs_options;

typedef struct bcs_plan bcs_plan; /* opaque; immutable after creation, except for the
                                     kernels that bcs_plan_autotune /
                                     bcs_multi_autotune choose */

/* Solver options of a plan (the kernel configuration choices of Section 3.2
 * and the solver of Section 3.1).  Fill `opt` with the defaults: FP64, Jacobi, J_GAMMA, lanes chosen by the
 * library, residual replacement on, 1 breakdown restart, inner_rtol 1e-4,
 * max_refine 10, refine_budget BCS_BUDGET_INNER, jit 1, autotune 1,
 * cell_order 1, shared_scalars 0, ilu_sweeps 0. */
void bcs_options_default(bcs_options* opt);

/* Create a plan: the shared sparsity pattern of every cell's Jacobian
 * (Section 2.2) and the kernels that solve one cell per workgroup slot
 * (Section 3.1).  The n x n pattern has nnz entries in CSR form (row_ptr[n+1],
 * col_idx[nnz], HOST int32 arrays) with row_ptr[0] = 0, row_ptr[n] = nnz,
 * non-decreasing row_ptr, strictly increasing columns in [0, n) within each
 * row, and (for BCS_J_GAMMA, Jacobi or ILU(0) preconditioning or
 * FP32_REFINE) every diagonal entry; n <= 255.  ILU(0) plans also need their
 * factor block (nnz + 3 doubles per cell slot) and the factorisation program
 * to fit a workgroup's LDS at some lane count, else BCS_ERR_UNSUPPORTED.  opt == NULL means defaults.  Allocates the plan's
 * device tables on the current HIP device (the plan must be used on that
 * device) and may compile kernels (hipRTC) and time them on a synthetic batch.
 * On error *out is set to NULL. */
int bcs_plan_create(int32_t n, int32_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                    const bcs_options* opt, bcs_plan** out);

/* Release a plan (the shared pattern of Section 2.2 and its kernels) and its
 * device tables (NULL is allowed).  The caller must
 * ensure no solve using it is still running. */
void bcs_plan_destroy(bcs_plan* plan);

/* Bytes of device workspace a solve of `ncells` cells with this plan needs
 * (forward, adjoint and the no-allocation variant alike): the work queue
 * (256 bytes), the cost-order sort state and 4 bytes per cell for the order.
 * Returns 0 only for a NULL plan or ncells < 0.  The cells of Section 3.2's
 * Block-cells arrangement are handed to persistent workgroups through this
 * queue instead of one block per cell. */
size_t bcs_workspace_bytes(const bcs_plan* plan, int64_t ncells);

/* Autotuner on the caller's data (the kernel configurations of Section 3.2,
 * chosen by measurement instead of fixed per mechanism): time the forward
 * solve of this batch with every lanes-per-cell layout that holds the pattern
 * (16, 32, 64 lanes per cell, i.e. 16, 8 or 4 cells per workgroup of four
 * waves) and keep the fastest in the plan, adjoint included.  Arguments as in
 * bcs_solve_batch (x/iters/resid/status serve as scratch and hold one solve's
 * outputs afterwards); allocates and frees its own workspace, synchronises the
 * device; *lanes_out (may be NULL) receives the chosen lanes per cell.  Not to
 * be called while solves with the plan run. */
int bcs_plan_autotune(bcs_plan* plan, int64_t ncells, const double* values, const double* gamma,
                      int64_t gamma_stride, const double* b, double rtol, int32_t maxit, double* x,
                      int32_t* iters, double* resid, int32_t* status, int32_t* lanes_out);

/* Shapes of the gather schedules of the specialised kernels (bit mask). */
#define BCS_SCHED_SPAN 1 /* the longest rows may span row slots 0 and 1 of one lane */
#define BCS_SCHED_DIAG 2 /* diagonal entries left out; the row sum starts from the diagonal term */

/* Matrices bcs_schedule_describe can describe (its `transpose` argument). */
#define BCS_PART_A 0       /* A */
#define BCS_PART_AT 1      /* A^T, as the adjoint solves it */
#define BCS_PART_LOWER 2   /* strict lower triangle (ILU(0) factor L_s) */
#define BCS_PART_UPPER 3   /* strict upper triangle (ILU(0) factor U_s) */

/* Describe, on the host (no device needed), the gather schedule the
 * specialised solve kernels use for a pattern: its rows dealt to row slots of
 * `lanes` lanes (16, 32 or 64) by decreasing length, each lane's entries step
 * after step (the sliced-ELL layout of the per-cell SpMV that Section 3.1's
 * solver performs, one row per thread there, several rows per lane here), for
 * the matrix named by `transpose` (BCS_PART_*: A, A^T, or the strict lower or
 * upper triangle of A, whose rows the ILU(0) kernel deals by their own
 * lengths; positions are those of the full pattern), with the schedule
 * shapes allowed by `shapes` (BCS_SCHED_* mask; the diagonal is left out
 * only if every row holds it, never for a triangle).  For tests and tuning.
 *   *steps          gather steps per lane
 *   *rows_per_lane  row slots per lane, ceil(n / lanes)
 *   *shape          the BCS_SCHED_* shapes used
 *   seg [rows_per_lane]             steps of each row slot, in order
 *   row [rows_per_lane * lanes]     row of slot j on lane l at j * lanes + l;
 *                                   -1 = none; -2 = slot 1 of a lane whose
 *                                   slot-0 row continues over slot 1's steps
 *   pos [steps * lanes]             CSR position (in the pattern as given) of
 *                                   the value at step s on lane l, at
 *                                   s * lanes + l; -1 = padding step
 *   col [steps * lanes]             column (row, for A^T) gathered at that step;
 *                                   n at a padding step (a zero spare element)
 * Each output may be NULL; the arrays must hold the sizes above (call once
 * with NULL arrays to learn steps).  Returns BCS_OK or an error code. */
int bcs_schedule_describe(int32_t n, int32_t nnz, const int32_t* row_ptr, const int32_t* col_idx, int32_t lanes,
                          int32_t transpose, int32_t shapes, int32_t* steps, int32_t* rows_per_lane,
                          int32_t* shape, int32_t* seg, int16_t* row, int32_t* pos, uint8_t* col);

/* Describe, on the host, the program by which the ILU(0) kernel factorises
 * one cell for a pattern (every row holding its diagonal) and lane count
 * (16, 32 or 64).  The cell's factor block holds the nnz values in CSR order
 * and three constants at positions nnz (0.0), nnz + 1 (1.0) and nnz + 2
 * (scratch).  Step st has widths[st] terms and runs one operation per lane:
 * its words (lanes head words, then widths[st] x lanes term words, lane
 * minor, steps one after another) give, per lane, head = target | divisor
 * << 16 and term = p | q << 16, and the operation is
 *   F[target] = (F[target] - sum over its terms of F[p] F[q]) / F[divisor].
 * Running the steps in order turns A into its ILU(0) factors (L strictly
 * below the diagonal, unit diagonal implied; U on and above it): the IKJ
 * elimination restricted to the pattern (Saad, Iterative Methods for Sparse
 * Linear Systems, Algorithm 10.4), per entry, the operations of one step
 * independent of each other.  For tests.
 *   *nsteps   steps
 *   widths    [nsteps] (may be NULL)
 *   *nwords   words (sum over steps of (1 + widths[st]) * lanes)
 *   words     [nwords] (may be NULL)
 * Call once with NULL arrays to learn the sizes.  Returns BCS_OK or an error
 * code (BCS_ERR_UNSUPPORTED if positions do not fit 16 bits). */
int bcs_ilu_describe(int32_t n, int32_t nnz, const int32_t* row_ptr, const int32_t* col_idx, int32_t lanes,
                     int32_t* nsteps, int32_t* widths, int32_t* nwords, uint32_t* words);

/* Describe the plan's launch configuration (the threads- and cells-per-block
 * choice of Section 3.2's Table 1, here per wavefront): lanes per cell, rows
 * per lane, schedule steps per lane, cells per workgroup.  Any output pointer
 * may be NULL. */
int bcs_plan_info(const bcs_plan* plan, int32_t* lanes_per_cell, int32_t* rows_per_lane,
                  int32_t* steps_per_lane, int32_t* cells_per_wg);

/* Solve (I - gamma_c J_c) x_c = b_c (or A_c x_c = b_c) for every cell c by
 * BiCGStab, stopping when the relative residual ||r||/||b|| is <= rtol and
 * confirming it on the true residual (Section 3.1's linear solve, one
 * workgroup-resident solve per cell, the whole batch in one kernel call with
 * no host reduction).
 *   values [ncells, nnz]  device, FP64: J (BCS_J_GAMMA) or A (BCS_A_DIRECT)
 *   gamma                 device, FP64: gamma of cell c is gamma[c*gamma_stride]
 *                         (gamma_stride 0 = one shared value); unused for A_DIRECT
 *   b [ncells, n]         device, FP64
 *   x0 [ncells, n]        device, FP64 initial guess, or NULL for x0 = 0.  A cell
 *                         whose initial true residual already meets rtol returns
 *                         x0 with 0 iterations.  Not with shared_scalars.
 *   rtol > 0, 1 <= maxit <= 1000000: the iteration budget of a cell
 *                         (FP32_REFINE: see refine_budget)
 *   x [ncells, n]         device, FP64 out: last iterate (also when not converged)
 *   iters [ncells]        device, int32 out: BiCGStab iterations (half-step exit
 *                         counts 1; FP32_REFINE: total inner iterations)
 *   resid [ncells]        device, FP64 out: true relative residual ||b-Ax||/||b||
 *                         recomputed in FP64 (0 when b = 0)
 *   status [ncells]       device, int32 out: BCS_CONVERGED .. BCS_NONFINITE
 *   refinements [ncells]  device, int32 out or NULL: FP32_REFINE inner solves
 *                         performed (0 for FP64)
 *   workspace             device, >= bcs_workspace_bytes(plan, ncells) bytes
 * The input arrays must not overlap the output arrays (x0 may equal x). */
int bcs_solve_batch(const bcs_plan* plan, int64_t ncells, const double* values, const double* gamma,
                    int64_t gamma_stride, const double* b, const double* x0, double rtol, int32_t maxit,
                    double* x, int32_t* iters, double* resid, int32_t* status, int32_t* refinements,
                    void* workspace, size_t workspace_bytes, void* stream);

/* Bytes of the library-owned scratch of bcs_solve_batch_noalloc (per GPU). */
#define BCS_NOALLOC_MAX_BYTES (4u << 20)

/* bcs_solve_batch for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * no workspace argument.  The solve's scratch (work queue, cost-order sort
 * state and order) lives in a library-owned device array of
 * BCS_NOALLOC_MAX_BYTES on every GPU the library runs on, held until the
 * process ends; the call allocates and frees nothing.  Limit:
 * bcs_workspace_bytes(plan, ncells) <= BCS_NOALLOC_MAX_BYTES, i.e. at most
 * 1,048,256 cells; a larger batch is rejected with BCS_ERR_UNSUPPORTED
 * before anything is launched.  Every call on one GPU shares that GPU's
 * array, which keeps the last call's contents (each call clears what must
 * start at zero itself, by a kernel on `stream`): calls that overlap on one
 * GPU (different streams or host threads without ordering) race and must be
 * serialised by the caller.  Arguments, outputs and errors otherwise as in
 * bcs_solve_batch; results are those of bcs_solve_batch. */
int bcs_solve_batch_noalloc(const bcs_plan* plan, int64_t ncells, const double* values, const double* gamma,
                            int64_t gamma_stride, const double* b, const double* x0, double rtol, int32_t maxit,
                            double* x, int32_t* iters, double* resid, int32_t* status, int32_t* refinements,
                            void* stream);

/* What the adjoint writes into grad_vals. */
#define BCS_GRAD_A 0      /* dL/dA on the pattern: -lambda_i x_j at entry (i, j) */
#define BCS_GRAD_VALUES 1 /* dL/d(values): in BCS_J_GAMMA mode dL/dJ = gamma_c lambda_i x_j
                             (A = I - gamma J); in BCS_A_DIRECT mode the same as BCS_GRAD_A */

/* Adjoint of the solve for a loss L(x), the reverse-mode derivative of the
 * linear solve in the BDF Newton step (Section 2.2): given the forward
 * solution x and g = dL/dx, solve A_c^T lambda_c = g_c by the same batched
 * BiCGStab run on the transposed pattern (same workgroup layout, FP64), then
 * write
 *   grad_b [ncells, n]       = lambda                                  (dL/db)
 *   grad_vals [ncells, nnz]  = per grad_kind (BCS_GRAD_A / BCS_GRAD_VALUES)
 *   grad_gamma [ncells]      = dL/dgamma_c = sum over entries (i, j) of
 *                              J_ij lambda_i x_j (BCS_J_GAMMA only; may be NULL;
 *                              must be NULL in BCS_A_DIRECT mode).  With
 *                              gamma_stride 0 the derivative with respect to the
 *                              shared gamma is the sum of these per-cell terms.
 * iters/resid/status describe the transposed solve.  Other arguments as in
 * bcs_solve_batch; x and g are device [ncells, n] FP64. */
/* (Not available for ILU(0) plans: BCS_ERR_UNSUPPORTED.) */
int bcs_solve_batch_adjoint(const bcs_plan* plan, int64_t ncells, const double* values,
                            const double* gamma, int64_t gamma_stride, const double* x, const double* g,
                            double rtol, int32_t maxit, int32_t grad_kind, double* grad_b, double* grad_vals,
                            double* grad_gamma, int32_t* iters, double* resid, int32_t* status,
                            void* workspace, size_t workspace_bytes, void* stream);

/* Bytes of device workspace bcs_solve_multi needs for these mechanisms: the
 * sum over mechanisms of bcs_workspace_bytes(plans[m], ncells[m]) (each part
 * 256-byte aligned).  Returns 0 on a bad argument. */
size_t bcs_multi_workspace_bytes(int32_t nmech, const bcs_plan* const* plans, const int64_t* ncells);

/* One persistent launch over several mechanisms (plans), each with its own
 * cells: workgroups pull cells from per-mechanism work queues, so a cell
 * slot that converges takes the next unsolved cell (the remainder kernel of
 * Section 3.2 and the fixed cells-per-block choices of Table 1 replaced by
 * work stealing).  Arrays are per mechanism m (host arrays of device
 * pointers, length nmech); semantics per cell as in bcs_solve_batch with
 * x0 = 0.  All plans must use BCS_FP64, jit = 1 and a Jacobi or no
 * preconditioner.  nmech <= 8.  The
 * mechanisms' LDS layouts must fit one workgroup together (64 KiB); a
 * combination that does not is rejected with BCS_ERR_UNSUPPORTED before
 * anything is compiled or launched. */
int bcs_solve_multi(int32_t nmech, const bcs_plan* const* plans, const int64_t* ncells,
                    const double* const* values, const double* const* gamma, const int64_t* gamma_stride,
                    const double* const* b, double rtol, int32_t maxit, double* const* x,
                    int32_t* const* iters, double* const* resid, int32_t* const* status, void* workspace,
                    size_t workspace_bytes, void* stream);

/* Autotuner of the one-launch form: choose every plan's lanes per cell for
 * the combined launch by timing bcs_solve_multi on the caller's batches
 * (coordinate descent: each mechanism in turn tries 16, 32 and 64 lanes with
 * the others held, for up to two passes; plans created with a fixed
 * lanes_per_cell keep it; mechanisms without cells are left as they are).
 * Every combination tried is compiled once (hipRTC, cached on disk like the
 * plans' kernels), so a first call can take seconds.  The choice is kept in
 * the plans (adjoint kernels included).  The combined kernel runs at the
 * occupancy of its most register-hungry mechanism, so the best lanes for it
 * can differ from each plan's best alone.  Arguments as in bcs_solve_multi,
 * on the null stream, with a workspace it allocates itself; the outputs serve
 * as scratch and hold one solve's results afterwards; synchronises the
 * device; lanes_out (may be NULL) receives nmech lane counts.  Not to be
 * called while solves with the plans run. */
int bcs_multi_autotune(int32_t nmech, bcs_plan* const* plans, const int64_t* ncells, const double* const* values,
                       const double* const* gamma, const int64_t* gamma_stride, const double* const* b,
                       double rtol, int32_t maxit, double* const* x, int32_t* const* iters, double* const* resid,
                       int32_t* const* status, int32_t* lanes_out);

/* ---- Mass-action rates and Jacobian on the device ----
 * The inputs of the solve for a mechanism of elementary reactions (the
 * per-cell rate equations of Section 2.1; Section 6 names moving the rest of
 * the BDF step onto the GPU as the next step).  Reaction r has reactants
 * reactants[2r] (required) and reactants[2r+1] (-1 = none; equal to the first
 * for A + A) and products products[2r], products[2r+1] (-1 = none).  It runs
 * at w_r = k_r y_a (one reactant) or (k_r y_a) y_b (two).  Per cell,
 *   f_i  = sum_r S_ir w_r                       (S_ir = products - reactants)
 *   J_ij = sum_r S_ir dw_r/dy_j  on the pattern (CSR order), with
 *          dw/dy_a = k_r (one reactant); k_r y_b, k_r y_a (a != b); 2 (k_r y_a) (a == b).
 * Every sum is taken over reactions in increasing order, one rounding per
 * term (S_ir times the rounded derivative or rate is exact). */
typedef struct bcs_mechanism bcs_mechanism; /* opaque, immutable */

/* Build a mechanism's gather tables for a pattern (HOST arrays: row_ptr[n+1],
 * col_idx[nnz] as in bcs_plan_create, reactants/products [nreact, 2] int32)
 * and copy them to the current device.  n < 65535.  BCS_ERR_PATTERN if the
 * pattern is malformed or lacks an entry (i, j) that a reaction's J needs
 * (every species i of the reaction against each of its reactants j);
 * BCS_ERR_ARG for species out of range.  Validation happens on the host,
 * before any device call.  On error *out is NULL. */
int bcs_mechanism_create(int32_t n, int32_t nnz, const int32_t* row_ptr, const int32_t* col_idx, int32_t nreact,
                         const int32_t* reactants, const int32_t* products, bcs_mechanism** out);

/* Release a mechanism (NULL allowed); no assembly may still be running. */
void bcs_mechanism_destroy(bcs_mechanism* mech);

/* f and J of every cell on `stream`:
 *   y [ncells, n]          device FP64 concentrations
 *   k                      device FP64 rate constants: k_r of cell c at
 *                          k[c * k_stride + r]; k_stride 0 = one set shared by
 *                          every cell, else >= nreact
 *   f [ncells, n]          device FP64 out, or NULL
 *   J [ncells, nnz]        device FP64 out (the values a J_GAMMA solve takes),
 *                          or NULL
 * Allocates nothing.  BCS_ERR_UNSUPPORTED if the mechanism's tables do not
 * fit a workgroup's LDS (64 KiB, about 9,000 reaction-entry terms). */
int bcs_assemble(const bcs_mechanism* mech, int64_t ncells, const double* y, const double* k, int64_t k_stride,
                 double* f, double* J, void* stream);

/* A plan for the mechanism's pattern whose forward solves take the cells'
 * concentrations instead of their Jacobian values: each cell's J is
 * assembled inside the solve kernel while the cell is staged (the sums and
 * roundings of bcs_assemble), so J never travels through device memory (the
 * paper's next step, the rest of the BDF step inside the Block-cells kernel,
 * Section 6).  The mechanism must outlive the plan.  Options as in
 * bcs_plan_create, limited to FP64, no or Jacobi preconditioning, J_GAMMA,
 * jit = 1, shared_scalars = 0 (else BCS_ERR_UNSUPPORTED; also when, at the
 * plan's lanes per cell, the solve's layout, the rate constants (within the
 * first 64 KiB) and the J term program, 8 bytes per lane for every term of
 * every schedule position, do not fit the device's LDS per workgroup, 160 KiB
 * on gfx950).  The plan also serves bcs_solve_batch, the adjoint and the
 * tuners like any other; bcs_plan_autotune keeps its mechanism kernel at the
 * chosen lanes. */
int bcs_plan_create_mech(const bcs_mechanism* mech, const bcs_options* opt, bcs_plan** out);

/* Solve (I - gamma_c J(y_c)) x_c = b_c for every cell, J assembled from the
 * concentrations y [ncells, n] (device FP64) and the rate constants k (device
 * FP64, k_r of cell c at k[c * k_stride + r]; k_stride 0 = one shared set,
 * else >= nreact), with a plan from bcs_plan_create_mech.  Results are
 * bitwise those of bcs_assemble followed by bcs_solve_batch with the same
 * plan; other arguments, outputs and errors as in bcs_solve_batch (no
 * refinements output). */
int bcs_solve_batch_mech(const bcs_plan* plan, int64_t ncells, const double* y, const double* k, int64_t k_stride,
                         const double* gamma, int64_t gamma_stride, const double* b, const double* x0, double rtol,
                         int32_t maxit, double* x, int32_t* iters, double* resid, int32_t* status, void* workspace,
                         size_t workspace_bytes, void* stream);

/* Debug aid for the persistent work queue (Section 3.2's remainder handling
 * replaced by work stealing): while `counts` (a device int32 array of at
 * least ncells zeros) is set, every forward, adjoint, mixed or ILU(0) solve
 * issued from this host thread with one mechanism increments counts[c] each
 * time it writes cell c's outputs, so a caller can check that every cell is
 * handed out exactly once.  NULL turns it off (the default).  Only kernels
 * compiled per pattern while the environment variable BCS_DEBUG_VISITS is
 * set (to anything but "0") at plan creation hold the counter, which costs
 * registers; other kernels ignore it.  Not for bcs_solve_multi. */
void bcs_debug_count_visits(int32_t* counts);

/* Description of the last error on this thread ("" if none).  Errors are
 * argument, pattern or runtime failures of a call, reported synchronously;
 * the numerical outcome of each cell's solve (Section 3.1's per-cell
 * convergence) is never an error but its status. */
const char* bcs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BCS_H */
