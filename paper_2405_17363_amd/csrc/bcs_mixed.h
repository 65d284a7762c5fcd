// Mixed-precision batched solve: FP32 inner BiCGStab inside FP64 iterative
// refinement, one cell per slot, same persistent work-queue structure as the
// FP64 kernel.
//
// Per cell (D = diag(A)):
//   Ahat = A D^-1 is formed in FP64 and held in VGPRs in FP32;
//   x = x0 (or 0), r = b - A x (FP64);
//   repeat while ||r||/||b|| > rtol, fewer than max_refine inner solves ran
//   and (budget per cell) fewer than maxit inner iterations over all inner
//   solves were spent:
//     solve Ahat d = float(r / ||r||) by FP32 BiCGStab to inner_rtol, within
//     maxit iterations (budget per inner solve) or the cell's remaining
//     budget (d0 = 0; an exact breakdown restarts once from the FP32 true
//     residual);
//     x_new = x + ||r|| D^-1 d (FP64); r_new = b - A x_new (FP64, with A
//     streamed again from memory, so the FP64 matrix never occupies VGPRs);
//     stop without accepting x_new if ||r_new|| >= ||r|| (stagnation).
// Outputs: x, iters = total inner iterations, refinements = inner solves,
// resid = ||b - A x||/||b|| in FP64, status.
#pragma once

#include "bcs_device.h"

namespace bcs {

template <class S>
__device__ __forceinline__ void mixed_body(const KParams& P) {
  using namespace dev;
  constexpr int LANES = S::LANES, RPL = S::RPL, KMAX = S::KMAX;
  constexpr int G = 64 / LANES;
  constexpr int NW = S::NW, PACK = S::PACK;
  const S sch(P.sched);
  extern __shared__ double lds[];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int gl = lane & (LANES - 1);
  const int grp = lane / LANES;
  double* xb = lds + wv * P.wxs + grp * P.xs;
  double* yb = lds + P.bbase + wv * P.wbs + grp * P.bs + P.yoff;
  const int n = P.n, nnz = P.nnz;

  uint32_t ad[NW];
  build_addr<PACK, KMAX, LANES>(ad, P.sched.col, lds_addr(xb), gl);
  if (gl == 0) xb[n] = 0.0;  // the spare element padding steps gather
  wave_sync();
  int rows[RPL];
#pragma unroll
  for (int j = 0; j < RPL; ++j) {
    const int rj = P.sched.row[j * LANES + gl];
    rows[j] = rj >= 0 ? rj : n;
  }
  int32_t* ent_lds = (int32_t*)(lds + P.tbase);
  for (int i = threadIdx.x; i < KMAX * LANES; i += kWgThreads) ent_lds[i] = P.sched.ent[i];
  __syncthreads();
  int dpos[RPL];
#pragma unroll
  for (int j = 0; j < RPL; ++j) dpos[j] = P.diag_pos[rows[j] < n ? rows[j] : 0] & kEntPosMask;

  float a32[KMAX];                      // Ahat = A D^-1 rounded to FP32
  double x64[RPL], r64[RPL], dg[RPL];   // FP64 iterate, residual, diag(A)
  float d[RPL], r[RPL], rh[RPL], p[RPL], v[RPL], t[RPL];  // FP32 inner state
  // Schedules without diagonal entries: the diagonal of Ahat in FP32 (that of
  // A, for the FP64 residual, is dg); 0 for padding rows.
  float dg32[RPL];
#pragma unroll
  for (int j = 0; j < RPL; ++j) dg32[j] = 0.f;
  // 1 on a lane whose slots 0 and 1 hold one long row
  double span64 = 0;
  if constexpr (S::FLAGS & kSchedSpan) span64 = (P.sched.row[LANES + gl] == kRowSpan) ? 1.0 : 0.0;
  const float span32 = (float)span64;
  double bn = 0, rn = 0, g = 0;
  float itol2 = 0, rho = 0, rho_prev = 1, alpha = 1, omega = 1;
  int it_in = 0, tot = 0, nref = 0, restarts_left = 0;
  bool first = true, active = false, dead = false;
  int phase = 0;  // 0: check / start an inner solve, 1: inner iterating, 2: refinement update
  int64_t cell = 0;
  int32_t held[kClaimGroup - 1];  // cells claimed and not yet started
#pragma unroll
  for (int q = 0; q < kClaimGroup - 1; ++q) held[q] = -1;
  held[0] = initial_held(P.queue, 0, P.ncells, wv, grp, 64 / LANES);  // no first claims without the counter

  auto finish = [&](int st, double res) {
#pragma unroll
    for (int j = 0; j < RPL; ++j)
      if (rows[j] < n) P.x[cell * n + rows[j]] = x64[j];
    if (gl == 0) {
      P.iters[cell] = tot;
      P.resid[cell] = res;
      P.status[cell] = st;
      if (P.refinements) P.refinements[cell] = nref;
#ifdef BCS_COUNT_VISITS
      if (P.visits) atomicAdd(P.visits + cell, 1);  // debug: outputs written per cell
#endif
    }
    active = false;
  };

  // out = b - A xin in FP64, with A's values streamed from memory (per step:
  // value position from the LDS schedule copy, the value, A = I - gamma J).
  auto residual64 = [&](const double (&xin)[RPL], double (&out)[RPL]) {
    const double* vals = P.values + cell * nnz;
    double av[KMAX];
#pragma unroll
    for (int s = 0; s < KMAX; ++s) {
      const int32_t e = ent_lds[s * LANES + gl];
      const double jv = vals[e & kEntPosMask];
      const double a = (P.kind == kJGamma) ? (((e & kEntDiag) ? 1.0 : 0.0) - g * jv) : jv;
      av[s] = (e & kEntPad) ? 0.0 : a;
    }
    double ax[RPL];
    sch.spmv(av, ad, xb, yb, gl, rows, xin, ax, dg, span64);
    const double* bc = P.b + cell * n;
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      const bool real = rows[j] < n;
      const double bj = bc[real ? rows[j] : 0];
      out[j] = (real ? bj : 0.0) - ax[j];
    }
  };

  // start the FP32 inner solve for the scaled residual r64 / rn
  auto start_inner = [&]() {
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      r[j] = (float)(r64[j] / rn);
      d[j] = 0.f;
      rh[j] = r[j];
      p[j] = 0.f;
      v[j] = 0.f;
    }
    const float ib2 = gsum<LANES>(ldot<RPL>(r, r));
    const float ibn = __builtin_sqrtf(ib2);
    const float tol = (float)P.inner_rtol * ibn;
    itol2 = tol * tol;
    rho = ib2;
    rho_prev = alpha = omega = 1.f;
    first = true;
    it_in = 0;
    restarts_left = 1;
  };

  // Take the next cell and stage it (sets dead when the queue is empty).
  auto claim_and_stage = [&]() {
    if (!claim_cell<false>(P.queue, P.order, P.ncells, grp * LANES, gl == 0, cell, held, wv, grp, 64 / LANES)) {
      dead = true;
    } else {
      const double* vals = P.values + cell * nnz;
      g = (P.kind == kJGamma) ? P.gamma[cell * P.gamma_stride] : 0.0;
      const double* bc = P.b + cell * n;
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        const bool real = rows[j] < n;
        const double bj = bc[real ? rows[j] : 0];
        const double dvj = vals[dpos[j]];
        dg[j] = (P.kind == kJGamma) ? 1.0 - g * dvj : dvj;
        r64[j] = real ? bj : 0.0;
        x64[j] = 0.0;
        const double dinv = real ? 1.0 / dg[j] : 0.0;
        xb[rows[j]] = dinv;  // D^-1 for the column scaling
        dg32[j] = (float)(dg[j] * dinv);
      }
      wave_sync();
      uint32_t ado[NW];
      opaque_copy<NW>(ad, ado);
#pragma unroll
      for (int s = 0; s < KMAX; ++s) {
        const int32_t e = ent_lds[s * LANES + gl];
        const double jv = vals[e & kEntPosMask];
        const double a = (P.kind == kJGamma) ? (((e & kEntDiag) ? 1.0 : 0.0) - g * jv) : jv;
        const double sc = lds_load<double>(step_addr<PACK>(ado, s));
        a32[s] = (e & kEntPad) ? 0.f : (float)(a * sc);
      }
      wave_sync();
      bn = __builtin_sqrt(gsum<LANES>(ldot<RPL>(r64, r64)));
      rn = bn;
      if (P.x0 != nullptr && finite(bn) && bn != 0.0) {
        // initial guess: refinement starts from x0 and r = b - A x0
        const double* x0c = P.x0 + cell * n;
#pragma unroll
        for (int j = 0; j < RPL; ++j) x64[j] = (rows[j] < n) ? x0c[rows[j]] : 0.0;
        residual64(x64, r64);
        rn = __builtin_sqrt(gsum<LANES>(ldot<RPL>(r64, r64)));
      }
      tot = 0;
      nref = 0;
      phase = 0;
      active = true;
      if (!finite(bn)) {
        finish(kNonfinite, __builtin_nan(""));
      } else if (bn == 0.0) {
        finish(kConverged, 0.0);
      }
    }
  };

  // Phase 0: stop the cell or start an inner solve (false: the cell ended).
  auto check_start = [&]() -> bool {
    if (!finite(rn)) {
      finish(kNonfinite, __builtin_nan(""));
      return false;
    }
    if (rn / bn <= P.rtol) {
      finish(kConverged, rn / bn);
      return false;
    }
    if (nref >= P.max_refine || (P.budget && tot >= P.maxit)) {
      finish(kMaxit, rn / bn);
      return false;
    }
    start_inner();
    return true;
  };

  // Phase 1: one FP32 BiCGStab iteration on Ahat d = r64 / rn; returns its
  // end (kConverged .. kNonfinite) or -1 to go on.
  auto inner_step = [&]() -> int {
    // one FP32 BiCGStab iteration on Ahat d = r64 / rn
    ++it_in;
    int ended = -1;
    if (!finite(rho)) {
      ended = kNonfinite;
    } else if (rho == 0.f) {
      ended = kBreakdown;
    } else {
      if (first) {
#pragma unroll
        for (int j = 0; j < RPL; ++j) p[j] = r[j];
        first = false;
      } else {
        const float beta = qdiv(rho * alpha, rho_prev * omega);
#pragma unroll
        for (int j = 0; j < RPL; ++j) p[j] = r[j] + beta * (p[j] - omega * v[j]);
      }
      sch.spmv(a32, ad, xb, yb, gl, rows, p, v, dg32, span32);
      const float sigma = gsum<LANES>(ldot<RPL>(rh, v));
      if (!finite(sigma)) {
        ended = kNonfinite;
      } else if (sigma == 0.f) {
        ended = kBreakdown;
      } else {
        alpha = qdiv(rho, sigma);
#pragma unroll
        for (int j = 0; j < RPL; ++j) r[j] = r[j] - alpha * v[j];  // r now holds s
        // t = Ahat s is formed before the half-step test so that ||s||^2,
        // (t, t) and (t, s) are reduced together (one reduction latency
        // instead of two; each sum is bitwise what its own reduction gives,
        // and t is discarded on a half-step exit)
        sch.spmv(a32, ad, xb, yb, gl, rows, r, t, dg32, span32);
        float red3[3] = {ldot<RPL>(r, r), ldot<RPL>(t, t), ldot<RPL>(t, r)};
        gsum_n<LANES>(red3);
        const float sn2 = red3[0];
        if (!finite(sn2)) {
          ended = kNonfinite;
        } else if (sn2 <= itol2) {
#pragma unroll
          for (int j = 0; j < RPL; ++j) d[j] = d[j] + alpha * p[j];
          ended = kConverged;
        } else {
          const float tt = red3[1], ts = red3[2];
          if (!finite(tt)) {
            ended = kNonfinite;
          } else if (tt == 0.f) {
            ended = kBreakdown;
          } else {
            omega = qdiv(ts, tt);
#pragma unroll
            for (int j = 0; j < RPL; ++j) {
              d[j] = d[j] + alpha * p[j] + omega * r[j];
              r[j] = r[j] - omega * t[j];
            }
            // ||r||^2 = ||s||^2 - omega (t, s) for r = s - omega t
            const float rn2 = sn2 - omega * ts;
            const float rho_next = gsum<LANES>(ldot<RPL>(rh, r));
            if (!finite(rn2)) {
              ended = kNonfinite;
            } else if (rn2 <= itol2) {
              ended = kConverged;
            } else if (omega == 0.f) {
              ended = kBreakdown;
            } else {
              rho_prev = rho;
              rho = rho_next;
            }
          }
        }
      }
    }
    return ended;
  };

  // After an inner iteration: 0 = go on iterating, 1 = the inner solve ended
  // (refinement update next), 2 = the cell ended.  maxit bounds each inner
  // solve, or (budget) the cell's inner iterations over all its refinements.
  auto inner_end = [&](int ended) -> int {
    const int used = P.budget ? tot : 0;
    if (ended < 0 && used + it_in >= P.maxit) ended = kMaxit;
    if (ended == kNonfinite) {
      tot += it_in;
      ++nref;
      finish(kNonfinite, __builtin_nan(""));
      return 2;
    }
    if (ended == kBreakdown && restarts_left > 0 && used + it_in < P.maxit) {
      // restart from the FP32 true residual of the scaled system
      --restarts_left;
      float ad32[RPL];
      sch.spmv(a32, ad, xb, yb, gl, rows, d, ad32, dg32, span32);
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        r[j] = (float)(r64[j] / rn) - ad32[j];
        rh[j] = r[j];
        p[j] = 0.f;
        v[j] = 0.f;
      }
      rho = gsum<LANES>(ldot<RPL>(r, r));
      rho_prev = alpha = omega = 1.f;
      first = true;
      return 0;
    }
    if (ended >= 0) {
      tot += it_in;
      ++nref;
      return 1;
    }
    return 0;
  };

  // Phase 2: the FP64 refinement x_new = x + ||r|| D^-1 d, accepted only if
  // the FP64 true residual decreases (false: the cell ended).
  auto refine = [&]() -> bool {
    double xn[RPL], rnv[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) xn[j] = x64[j] + rn * ((double)d[j] / dg[j]);
    residual64(xn, rnv);
    const double rnn = __builtin_sqrt(gsum<LANES>(ldot<RPL>(rnv, rnv)));
    if (!(rnn < rn)) {
      if (finite(rnn))
        finish(kMaxit, rn / bn);
      else
        finish(kNonfinite, __builtin_nan(""));
      return false;
    }
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      x64[j] = xn[j];
      r64[j] = rnv[j];
    }
    rn = rnn;
    return true;
  };

  if constexpr (G == 1) {
    // One cell per wave: every decision is the wave's, so the phases are
    // plain nested loops (the inner solve's iterations back to back), with
    // the loop conditions in scalar registers.
    for (;;) {
      claim_and_stage();
      if (__builtin_amdgcn_readfirstlane((int)dead)) break;
      if (!__builtin_amdgcn_readfirstlane((int)active)) continue;
      while (__builtin_amdgcn_readfirstlane((int)check_start())) {
        int e;
        do {
          e = __builtin_amdgcn_readfirstlane(inner_end(inner_step()));
        } while (e == 0);
        if (e == 2 || !__builtin_amdgcn_readfirstlane((int)refine())) break;
      }
    }
  } else {
    // Several cells per wave, each in its own phase.
    for (;;) {
      if (!active && !dead) claim_and_stage();
      if (__ballot(!dead) == 0ull) break;
      if (!active) continue;
      if (phase == 0) {
        if (!check_start()) continue;
        phase = 1;
      }
      if (phase == 1) {
        const int e = inner_end(inner_step());
        if (e == 2) continue;
        if (e == 1) phase = 2;
      }
      if (phase == 2) {
        if (!refine()) continue;
        phase = 0;
      }
    }
  }
}

}  // namespace bcs
