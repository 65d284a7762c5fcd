// Host side of the library: pattern validation, schedule construction, plan
// objects and the C-ABI entry points declared in include/bcs.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "bcs_internal.h"

namespace bcs {
const Variant* variants_l16(int* count);
const Variant* variants_l32(int* count);
const Variant* variants_l64(int* count);
}  // namespace bcs

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(BCS_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Host form of a schedule (see DevSchedule).
struct HostSchedule {
  int lanes = 0, rpl = 0, ksteps = 0;
  std::vector<int32_t> ent;
  std::vector<uint8_t> col;
  std::vector<int16_t> row;
  uint64_t flush[2] = {0, 0};
};

// Deal the rows of a CSR matrix (rp, ci; entry k stores value position
// pos[k]) to `rpl` slots of `lanes` lanes, longest rows first, and list each
// lane's entries slot after slot.  Slot j spans the same LEN_j steps on every
// lane, LEN_j = longest row in the slot (at least 1); shorter rows and absent
// rows are padded with entries of value 0 that gather column 0, and the last
// slot is extended so that every lane runs exactly kmax steps.
HostSchedule build_schedule(int n, const std::vector<int>& rp, const std::vector<int>& ci,
                            const std::vector<int>& pos, int lanes, int rpl, int kmax) {
  HostSchedule S;
  S.lanes = lanes;
  S.rpl = rpl;
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int u, int v) { return (rp[u + 1] - rp[u]) > (rp[v + 1] - rp[v]); });
  S.row.assign((size_t)rpl * lanes, -1);
  std::vector<int> len(rpl, 1);
  for (int j = 0; j < rpl; ++j)
    for (int l = 0; l < lanes; ++l) {
      const int q = j * lanes + l;
      if (q < n) {
        const int i = order[q];
        S.row[q] = (int16_t)i;
        len[j] = std::max(len[j], rp[i + 1] - rp[i]);
      }
    }
  int ks = 0;
  for (int j = 0; j < rpl; ++j) ks += len[j];
  S.ksteps = ks;
  if (ks > kmax) return S;  // does not fit; the caller checks ksteps
  // pad the last slot so that every lane runs exactly kmax steps
  len[rpl - 1] += kmax - ks;
  ks = kmax;
  S.ksteps = ks;
  S.ent.assign((size_t)ks * lanes, bcs::kEntPad);
  S.col.assign((size_t)ks * lanes, 0);
  int s0 = 0;
  for (int j = 0; j < rpl; ++j) {
    for (int l = 0; l < lanes; ++l) {
      const int i = S.row[j * lanes + l];
      if (i < 0) continue;
      for (int t = 0; t < rp[i + 1] - rp[i]; ++t) {
        const int k = rp[i] + t;
        const size_t at = (size_t)(s0 + t) * lanes + l;
        S.ent[at] = pos[k] | (ci[k] == i ? bcs::kEntDiag : 0);
        S.col[at] = (uint8_t)ci[k];
      }
    }
    const int last = s0 + len[j] - 1;
    if (last < 64)
      S.flush[0] |= 1ull << last;
    else
      S.flush[1] |= 1ull << (last - 64);
    s0 += len[j];
  }
  return S;
}

struct DeviceSchedule {
  bcs::DevSchedule d;
  const bcs::Variant* var = nullptr;
  int max_blocks = 0;  // resident workgroups per CU for this variant
  void* buf = nullptr;
};

}  // namespace

struct bcs_plan {
  int n = 0, nnz = 0;
  int device = 0;
  int num_cu = 0;
  bcs_options opt{};
  std::vector<int> rp, ci;
  DeviceSchedule fwd, adj;
  int32_t* diag_pos = nullptr;
  int16_t* coo_row = nullptr;
  int16_t* coo_col = nullptr;
  unsigned long long* queue = nullptr;  // [0..1] forward solves, [2..3] adjoint solves
};

namespace {

const bcs::Variant* all_variants(int* count) {
  static std::vector<bcs::Variant> all;
  static std::once_flag once;
  std::call_once(once, [] {
    int c = 0;
    const bcs::Variant* v = bcs::variants_l16(&c);
    all.insert(all.end(), v, v + c);
    v = bcs::variants_l32(&c);
    all.insert(all.end(), v, v + c);
    v = bcs::variants_l64(&c);
    all.insert(all.end(), v, v + c);
  });
  *count = (int)all.size();
  return all.data();
}

// Smallest compiled variant for `lanes` that holds the pattern; builds the
// schedule for it.  Returns nullptr if none fits.
const bcs::Variant* pick_variant(int n, const std::vector<int>& rp, const std::vector<int>& ci,
                                 const std::vector<int>& pos, int lanes, HostSchedule* out) {
  int nv = 0;
  const bcs::Variant* vs = all_variants(&nv);
  const int need_rpl = (n + lanes - 1) / lanes;
  const bcs::Variant* best = nullptr;
  for (int q = 0; q < nv; ++q) {
    const bcs::Variant& v = vs[q];
    if (v.lanes != lanes || v.rpl < need_rpl) continue;
    HostSchedule S = build_schedule(n, rp, ci, pos, lanes, v.rpl, v.kmax);
    if (S.ksteps > v.kmax) continue;
    if (!best || v.rpl < best->rpl || (v.rpl == best->rpl && v.kmax < best->kmax)) {
      best = &v;
      *out = std::move(S);
    }
  }
  return best;
}

int upload_schedule(const HostSchedule& S, const bcs::Variant* var, DeviceSchedule* D) {
  const size_t ne = S.ent.size();
  const size_t bytes = ne * 4 + ne + S.row.size() * 2 + 64;
  void* buf = nullptr;
  HIP_TRY(hipMalloc(&buf, bytes));
  D->buf = buf;
  char* p = (char*)buf;
  HIP_TRY(hipMemcpy(p, S.ent.data(), ne * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p + ne * 4, S.row.data(), S.row.size() * 2, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p + ne * 4 + S.row.size() * 2, S.col.data(), ne, hipMemcpyHostToDevice));
  D->d.ent = (const int32_t*)p;
  D->d.row = (const int16_t*)(p + ne * 4);
  D->d.col = (const uint8_t*)(p + ne * 4 + S.row.size() * 2);
  D->d.ksteps = S.ksteps;
  D->d.rpl = S.rpl;
  D->d.flush[0] = S.flush[0];
  D->d.flush[1] = S.flush[1];
  D->var = var;
  return BCS_OK;
}

// LDS layout of one cell slot, in doubles: the SpMV operand (n values plus
// a spare element that padding rows write to), for the adjoint a second
// n-vector, then the SpMV result block (RPL x LANES).  The stride is padded so
// that the slots of a wave start on different LDS banks.
struct SlotLayout {
  int stride, xoff2, yoff;
};

SlotLayout slot_layout(int n, int lanes, int rpl, int adjoint) {
  SlotLayout L;
  const int xn = ((n + 1 + 7) / 8) * 8;
  L.xoff2 = xn;
  L.yoff = adjoint ? 2 * xn : xn;
  const int used = L.yoff + rpl * lanes;
  L.stride = ((used + 31) / 32) * 32 + 8;
  return L;
}

size_t slot_lds_bytes(const bcs::Variant* v, int n, int adjoint) {
  return (size_t)bcs::kWavesPerWg * (64 / v->lanes) * slot_layout(n, v->lanes, v->rpl, adjoint).stride *
         sizeof(double);
}

int occupancy(const bcs::Variant* v, int n, int adjoint, int* blocks) {
  // gather addresses are 16-bit LDS byte addresses
  if (slot_lds_bytes(v, n, adjoint) > 65536)
    return fail(BCS_ERR_UNSUPPORTED, "workgroup LDS of %zu bytes exceeds 64 KiB", slot_lds_bytes(v, n, adjoint));
  int nb = 0;
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, v->fp64_kernel, bcs::kWgThreads,
                                                       slot_lds_bytes(v, n, adjoint)));
  *blocks = std::max(nb, 1);
  return BCS_OK;
}

void release(bcs_plan* p) {
  if (!p) return;
  int cur = 0;
  if (hipGetDevice(&cur) == hipSuccess && cur != p->device) (void)hipSetDevice(p->device);
  if (p->fwd.buf) (void)hipFree(p->fwd.buf);
  if (p->adj.buf) (void)hipFree(p->adj.buf);
  if (p->diag_pos) (void)hipFree(p->diag_pos);
  if (p->coo_row) (void)hipFree(p->coo_row);
  if (p->queue) (void)hipFree(p->queue);
  if (cur != p->device) (void)hipSetDevice(cur);
  delete p;
}

}  // namespace

extern "C" {

const char* bcs_last_error(void) { return g_err.c_str(); }

void bcs_options_default(bcs_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = BCS_FP64;
  o->precond = BCS_PRECOND_JACOBI;
  o->matrix_kind = BCS_J_GAMMA;
  o->lanes_per_cell = 0;
  o->residual_replacement = 1;
  o->breakdown_restarts = 1;
  o->inner_rtol = 1e-4;
  o->max_refine = 10;
}

int bcs_plan_create(int32_t n, int32_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                    const bcs_options* opt, bcs_plan** out) {
  g_err.clear();
  if (!out) return fail(BCS_ERR_ARG, "out is NULL");
  *out = nullptr;
  bcs_options o;
  bcs_options_default(&o);
  if (opt) o = *opt;
  if (n <= 0) return fail(BCS_ERR_ARG, "n must be positive (got %d)", n);
  if (nnz < 1) return fail(BCS_ERR_ARG, "nnz must be at least 1 (got %d)", nnz);
  if (!row_ptr || (nnz > 0 && !col_idx)) return fail(BCS_ERR_ARG, "row_ptr/col_idx is NULL");
  if (o.precision != BCS_FP64 && o.precision != BCS_FP32_REFINE)
    return fail(BCS_ERR_ARG, "unknown precision %d", o.precision);
  if (o.precond != BCS_PRECOND_NONE && o.precond != BCS_PRECOND_JACOBI)
    return fail(BCS_ERR_ARG, "unknown preconditioner %d", o.precond);
  if (o.matrix_kind != BCS_J_GAMMA && o.matrix_kind != BCS_A_DIRECT)
    return fail(BCS_ERR_ARG, "unknown matrix kind %d", o.matrix_kind);
  if (o.lanes_per_cell != 0 && o.lanes_per_cell != 16 && o.lanes_per_cell != 32 && o.lanes_per_cell != 64)
    return fail(BCS_ERR_ARG, "lanes_per_cell must be 0, 16, 32 or 64 (got %d)", o.lanes_per_cell);
  if (o.residual_replacement != 0 && o.residual_replacement != 1)
    return fail(BCS_ERR_ARG, "residual_replacement must be 0 or 1");
  if (o.breakdown_restarts < 0 || o.breakdown_restarts > 1000)
    return fail(BCS_ERR_ARG, "breakdown_restarts must be in [0, 1000]");
  if (o.precision == BCS_FP32_REFINE && (!(o.inner_rtol > 0.0 && o.inner_rtol < 1.0) || o.max_refine < 1))
    return fail(BCS_ERR_ARG, "FP32_REFINE needs 0 < inner_rtol < 1 and max_refine >= 1");
  for (int i = 0; i < 7; ++i)
    if (o.reserved[i] != 0) return fail(BCS_ERR_ARG, "reserved option fields must be zero");

  // pattern
  if (row_ptr[0] != 0) return fail(BCS_ERR_PATTERN, "row_ptr[0] must be 0");
  if (row_ptr[n] != nnz) return fail(BCS_ERR_PATTERN, "row_ptr[n] = %d but nnz = %d", row_ptr[n], nnz);
  std::vector<int> diag(n, -1);
  for (int i = 0; i < n; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) return fail(BCS_ERR_PATTERN, "row_ptr decreases at row %d", i);
  for (int i = 0; i < n; ++i) {
    for (int k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const int c = col_idx[k];
      if (c < 0 || c >= n) return fail(BCS_ERR_PATTERN, "column %d out of range in row %d", c, i);
      if (k > row_ptr[i] && c <= col_idx[k - 1])
        return fail(BCS_ERR_PATTERN, "columns of row %d are not strictly increasing", i);
      if (c == i) diag[i] = k;
    }
  }
  const bool need_diag = o.matrix_kind == BCS_J_GAMMA || o.precond == BCS_PRECOND_JACOBI ||
                         o.precision == BCS_FP32_REFINE;
  if (need_diag)
    for (int i = 0; i < n; ++i)
      if (diag[i] < 0) return fail(BCS_ERR_PATTERN, "row %d has no diagonal entry", i);
  if (n > 256) return fail(BCS_ERR_UNSUPPORTED, "n = %d exceeds the supported 256 rows per cell", n);

  bcs_plan* p = new bcs_plan();
  p->n = n;
  p->nnz = nnz;
  p->opt = o;
  p->rp.assign(row_ptr, row_ptr + n + 1);
  p->ci.assign(col_idx, col_idx + nnz);
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return fail(BCS_ERR_HIP, "no HIP device");
  }
  if (hipDeviceGetAttribute(&p->num_cu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess) {
    delete p;
    return fail(BCS_ERR_HIP, "cannot query the compute unit count");
  }

  // A and A^T patterns with value positions
  std::vector<int> pos(nnz);
  for (int k = 0; k < nnz; ++k) pos[k] = k;
  std::vector<int> trp(n + 1, 0), tci(nnz), tpos(nnz);
  for (int k = 0; k < nnz; ++k) trp[p->ci[k] + 1]++;
  for (int j = 0; j < n; ++j) trp[j + 1] += trp[j];
  {
    std::vector<int> fill(trp.begin(), trp.end() - 1);
    for (int i = 0; i < n; ++i)
      for (int k = p->rp[i]; k < p->rp[i + 1]; ++k) {
        const int q = fill[p->ci[k]]++;
        tci[q] = i;
        tpos[q] = k;
      }
  }

  // lanes per cell: fewest wave-steps per cell among the variants that fit
  HostSchedule fs, as;
  const bcs::Variant* fv = nullptr;
  const bcs::Variant* av = nullptr;
  double best_cost = 1e300;
  const int cand[3] = {16, 32, 64};
  for (int L : cand) {
    if (o.lanes_per_cell != 0 && o.lanes_per_cell != L) continue;
    HostSchedule f1, a1;
    const bcs::Variant* v1 = pick_variant(n, p->rp, p->ci, pos, L, &f1);
    const bcs::Variant* v2 = pick_variant(n, trp, tci, tpos, L, &a1);
    if (!v1 || !v2) continue;
    const double cost = (double)f1.ksteps * L / 64.0 + 0.25 * v1->rpl;
    if (cost < best_cost) {
      best_cost = cost;
      fv = v1;
      av = v2;
      fs = std::move(f1);
      as = std::move(a1);
    }
  }
  if (!fv) {
    release(p);
    return fail(BCS_ERR_UNSUPPORTED, "no compiled kernel variant holds this pattern (n = %d, nnz = %d)", n, nnz);
  }
  int rc = upload_schedule(fs, fv, &p->fwd);
  if (rc == BCS_OK) rc = upload_schedule(as, av, &p->adj);
  if (rc == BCS_OK) rc = occupancy(fv, n, 0, &p->fwd.max_blocks);
  if (rc == BCS_OK) rc = occupancy(av, n, 1, &p->adj.max_blocks);
  if (rc != BCS_OK) {
    release(p);
    return rc;
  }
  std::vector<int16_t> crow(std::max(nnz, 1)), ccol(std::max(nnz, 1));
  for (int i = 0; i < n; ++i)
    for (int k = p->rp[i]; k < p->rp[i + 1]; ++k) {
      crow[k] = (int16_t)i;
      ccol[k] = (int16_t)p->ci[k];
    }
  for (int i = 0; i < n; ++i) diag[i] = std::max(diag[i], 0);  // absent diagonal: never read, keep in bounds
  hipError_t e = hipMalloc((void**)&p->diag_pos, sizeof(int32_t) * n);
  if (e == hipSuccess) e = hipMemcpy(p->diag_pos, diag.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc((void**)&p->coo_row, sizeof(int16_t) * 2 * crow.size());
  if (e == hipSuccess) {
    p->coo_col = p->coo_row + crow.size();
    e = hipMemcpy(p->coo_row, crow.data(), sizeof(int16_t) * crow.size(), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMemcpy(p->coo_col, ccol.data(), sizeof(int16_t) * ccol.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc((void**)&p->queue, 4 * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMemset(p->queue, 0, 4 * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    release(p);
    return fail(BCS_ERR_HIP, "plan allocation: %s", hipGetErrorString(e));
  }
  *out = p;
  return BCS_OK;
}

void bcs_plan_destroy(bcs_plan* plan) { release(plan); }

int bcs_plan_info(const bcs_plan* p, int32_t* lanes, int32_t* rpl, int32_t* steps, int32_t* cells_per_wg) {
  if (!p) return fail(BCS_ERR_ARG, "plan is NULL");
  if (lanes) *lanes = p->fwd.var->lanes;
  if (rpl) *rpl = p->fwd.d.rpl;
  if (steps) *steps = p->fwd.d.ksteps;
  if (cells_per_wg) *cells_per_wg = bcs::kWavesPerWg * (64 / p->fwd.var->lanes);
  return BCS_OK;
}

static int check_common(const bcs_plan* p, int64_t ncells, const double* values, const double* gamma,
                        int64_t gamma_stride, double rtol, int32_t maxit) {
  if (!p) return fail(BCS_ERR_ARG, "plan is NULL");
  if (ncells < 0) return fail(BCS_ERR_ARG, "ncells must be >= 0");
  if (ncells > ((int64_t)1 << 40)) return fail(BCS_ERR_ARG, "ncells too large");
  if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(BCS_ERR_ARG, "rtol must be positive and finite");
  if (maxit < 1 || maxit > 1000000) return fail(BCS_ERR_ARG, "maxit must be in [1, 1000000]");
  if (ncells > 0 && !values && p->nnz > 0) return fail(BCS_ERR_ARG, "values is NULL");
  if (p->opt.matrix_kind == BCS_J_GAMMA) {
    if (ncells > 0 && !gamma) return fail(BCS_ERR_ARG, "gamma is NULL");
    if (gamma_stride < 0) return fail(BCS_ERR_ARG, "gamma_stride must be >= 0");
  }
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess || cur != p->device)
    return fail(BCS_ERR_ARG, "the plan belongs to device %d, current device is %d", p->device, cur);
  return BCS_OK;
}

static bcs::KParams base_params(const bcs_plan* p, int64_t ncells, const double* values, const double* gamma,
                                int64_t gamma_stride, double rtol, int32_t maxit) {
  bcs::KParams P{};
  P.ncells = ncells;
  P.n = p->n;
  P.nnz = p->nnz;
  P.values = values;
  P.gamma = gamma;
  P.gamma_stride = gamma_stride;
  P.rtol = rtol;
  P.maxit = maxit;
  P.precond = p->opt.precond;
  P.kind = p->opt.matrix_kind;
  P.rr = p->opt.residual_replacement;
  P.brs = p->opt.breakdown_restarts;
  P.inner_rtol = p->opt.inner_rtol;
  P.max_refine = p->opt.max_refine;
  P.diag_pos = p->diag_pos;
  P.coo_row = p->coo_row;
  P.coo_col = p->coo_col;
  return P;
}

static int grid_for(const bcs_plan* p, const DeviceSchedule& D, int64_t ncells) {
  const int64_t cells_per_wg = (int64_t)bcs::kWavesPerWg * (64 / D.var->lanes);
  const int64_t need = (ncells + cells_per_wg - 1) / cells_per_wg;
  const int64_t cap = (int64_t)D.max_blocks * p->num_cu;
  return (int)std::max<int64_t>(1, std::min(need, cap));
}

int bcs_solve_batch(const bcs_plan* p, int64_t ncells, const double* values, const double* gamma,
                    int64_t gamma_stride, const double* b, double rtol, int32_t maxit, double* x, int32_t* iters,
                    double* resid, int32_t* status, int32_t* refinements, void* stream) {
  g_err.clear();
  int rc = check_common(p, ncells, values, gamma, gamma_stride, rtol, maxit);
  if (rc != BCS_OK) return rc;
  if (ncells == 0) return BCS_OK;
  if (!b || !x || !iters || !resid || !status) return fail(BCS_ERR_ARG, "b/x/iters/resid/status is NULL");
  if (p->opt.precision != BCS_FP64) return fail(BCS_ERR_UNSUPPORTED, "FP32_REFINE is not available yet");
  bcs::KParams P = base_params(p, ncells, values, gamma, gamma_stride, rtol, maxit);
  P.b = b;
  P.x = x;
  P.iters = iters;
  P.resid = resid;
  P.status = status;
  P.refinements = refinements;
  P.sched = p->fwd.d;
  P.adjoint = 0;
  {
    const SlotLayout L = slot_layout(p->n, p->fwd.var->lanes, p->fwd.var->rpl, 0);
    P.xs = L.stride;
    P.xoff2 = L.xoff2;
    P.yoff = L.yoff;
  }
  P.queue = p->queue;
  const int grid = grid_for(p, p->fwd, ncells);
  P.total_waves = grid * bcs::kWavesPerWg;
  hipError_t e = p->fwd.var->fp64(P, grid, (hipStream_t)stream);
  if (e != hipSuccess) return fail(BCS_ERR_HIP, "solve launch: %s", hipGetErrorString(e));
  return BCS_OK;
}

int bcs_solve_batch_adjoint(const bcs_plan* p, int64_t ncells, const double* values, const double* gamma,
                            int64_t gamma_stride, const double* x, const double* g, double rtol, int32_t maxit,
                            double* grad_b, double* grad_A, int32_t* iters, double* resid, int32_t* status,
                            void* stream) {
  g_err.clear();
  int rc = check_common(p, ncells, values, gamma, gamma_stride, rtol, maxit);
  if (rc != BCS_OK) return rc;
  if (ncells == 0) return BCS_OK;
  if (!x || !g || !grad_b || !iters || !resid || !status || (!grad_A && p->nnz > 0))
    return fail(BCS_ERR_ARG, "x/g/grad_b/grad_A/iters/resid/status is NULL");
  bcs::KParams P = base_params(p, ncells, values, gamma, gamma_stride, rtol, maxit);
  P.b = g;
  P.xin = x;
  P.x = grad_b;
  P.grad_a = grad_A;
  P.iters = iters;
  P.resid = resid;
  P.status = status;
  P.refinements = nullptr;
  P.sched = p->adj.d;
  P.adjoint = 1;
  {
    const SlotLayout L = slot_layout(p->n, p->adj.var->lanes, p->adj.var->rpl, 1);
    P.xs = L.stride;
    P.xoff2 = L.xoff2;
    P.yoff = L.yoff;
  }
  P.queue = p->queue + 2;
  const int grid = grid_for(p, p->adj, ncells);
  P.total_waves = grid * bcs::kWavesPerWg;
  hipError_t e = p->adj.var->fp64(P, grid, (hipStream_t)stream);
  if (e != hipSuccess) return fail(BCS_ERR_HIP, "adjoint launch: %s", hipGetErrorString(e));
  return BCS_OK;
}

int bcs_solve_multi(int32_t nmech, const bcs_plan* const* plans, const int64_t* ncells,
                    const double* const* values, const double* const* gamma, const int64_t* gamma_stride,
                    const double* const* b, double rtol, int32_t maxit, double* const* x, int32_t* const* iters,
                    double* const* resid, int32_t* const* status, void* stream) {
  (void)nmech; (void)plans; (void)ncells; (void)values; (void)gamma; (void)gamma_stride; (void)b; (void)rtol;
  (void)maxit; (void)x; (void)iters; (void)resid; (void)status; (void)stream;
  return fail(BCS_ERR_UNSUPPORTED, "bcs_solve_multi is not available yet");
}

}  // extern "C"
