// Host-side internal definitions: the registry of precompiled kernel variants.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bcs.h"
#include "bcs_kdefs.h"

#ifdef __cplusplus
#include <vector>
#endif

// A mass-action mechanism on a pattern (bcs_mechanism_create): host copies of
// the pattern and the device gather tables of its rates and Jacobian.
struct bcs_mechanism {
  int n = 0, nnz = 0, R = 0;
  int device = 0;
  int num_cu = 0;
  int nj = 0, nf = 0;  // J and f terms
  std::vector<int> rp, ci;
  std::vector<int32_t> htab;  // host copy of the device tables (same word offsets)
  int jofs_at = 0, jterm_at = 0;  // word offsets of jofs and jterm in htab
  // device tables (one allocation): jofs [nnz + 1], jterm [nj] (2 words each),
  // fofs [n + 1], fterm [nf] (2 words each), reac [2 R]
  int32_t* buf = nullptr;
  int32_t* jofs = nullptr;
  int32_t* jterm = nullptr;
  int32_t* fofs = nullptr;
  int32_t* fterm = nullptr;
  int32_t* reac = nullptr;
  size_t table_words = 0;
};

namespace bcs {

static_assert(kConverged == BCS_CONVERGED && kMaxit == BCS_MAXIT && kBreakdown == BCS_BREAKDOWN &&
                  kNonfinite == BCS_NONFINITE,
              "status codes");
static_assert(kJGamma == BCS_J_GAMMA && kADirect == BCS_A_DIRECT, "matrix kinds");

// The library's thread-local error message (bcs_last_error): set it and
// return `code`, or clear it.
int set_error(int code, const char* msg);
void clear_error();

// Precompiled variants: (lanes per cell, row slots per lane, max steps per
// lane), with the slot segment boundaries read at run time.
using LaunchFn = hipError_t (*)(const KParams&, int grid, hipStream_t stream);

struct Variant {
  int lanes, rpl, kmax;
  LaunchFn fp64;
  LaunchFn mixed;
  const void* fp64_kernel;  // for occupancy queries
};

const Variant* variants_l16(int* count);
const Variant* variants_l32(int* count);
const Variant* variants_l64(int* count);

// Kernels specialised for one pattern's exact slot segments, compiled at
// plan creation with hipRTC (bcs_jit.cpp).
struct JitKernel {
  hipFunction_t fn = nullptr;
  int max_blocks = 0;   // resident workgroups per CU
  int scratch = 0;      // private (spill) bytes per lane
};

// Compile (or fetch from the cache) a solve kernel -- body "fp64_body" or
// "mixed_body" -- for `lanes` lanes per cell, schedule shape `flags`
// (kSchedSpan / kSchedDiag) and slot segment lengths seg[0..rpl); grouped:
// the FP64 forward body with one wave's cells solved as one system.  Returns
// BCS_OK or an error code with the message in `err`.
int jit_kernel(const char* body, int adjoint, int grouped, int lanes, int flags, const int* seg, int rpl,
               int waves_per_eu, size_t lds_bytes, JitKernel* out, char* err, size_t errlen,
               const std::vector<int>* mech_terms = nullptr, int wg_waves = kWavesPerWg);

// Prologue of every solve (bcs_order.hip), on `stream`: zero the work queue
// (kQueueWords words; the claim counter, word 0, set to qstart) and, when `order` is not null, fill order[0, ncells)
// with the cell indices sorted by a bucket of gamma[c * stride], largest
// first (state: kOrderStateWords words of scratch).
hipError_t launch_solve_prologue(unsigned long long* queue, unsigned long long qstart, const double* gamma,
                                 int64_t stride, int64_t ncells, uint32_t* state, int32_t* order, hipStream_t stream);

// The ILU(0) kernel for one pattern: schedules of A, L_s and U_s (flags,
// segment lengths, rows per lane each) and the factorisation program's step
// widths; waves_per_eu > 0 adds that launch bound.
int jit_ilu_kernel(int lanes, const int* flags, const int* const* seg, const int* rpl, int nnz,
                   const int* widths, int nstep, int waves_per_eu, size_t lds_bytes, JitKernel* out, char* err,
                   size_t errlen);

// The multi-mechanism kernel for mechanisms with the given layouts, in order.
int jit_multi_kernel(int nmech, const int* lanes, const int* flags, const int* const* seg, const int* rpl,
                     size_t lds_bytes, JitKernel* out, char* err, size_t errlen);

}  // namespace bcs
