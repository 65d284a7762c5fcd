// ILU(0)-preconditioned batched Block-cells BiCGStab (FP64, forward solves).
//
// Right preconditioning with M = L U, the incomplete LU factors of A on A's
// own sparsity pattern (ILU(0)).  The paper names a preconditioner as the
// most promising next optimisation of its solver (Section 5.2); because all
// cells share one pattern, everything symbolic (the elimination's dependency
// levels, the gather schedules of the factors) is computed once per plan on
// the host, and only the numeric factorisation runs per cell.
//
// Per cell, when a slot takes it:
//   1. A = I - gamma J is formed in the slot's LDS factor block (CSR order),
//      and the SpMV values of A are taken from it into registers;
//   2. the factor block is overwritten with L (strict lower part; unit
//      diagonal implied) and U (diagonal and upper part).  Entry (i, j)
//      becomes a_ij - sum_k l_ik u_kj over k < min(i, j) with (i, k) and
//      (k, j) in the pattern, in increasing k, then divided by u_jj when
//      i > j.  This is the IKJ elimination restricted to the pattern (Saad,
//      Iterative Methods for Sparse Linear Systems, Algorithm 10.4) written
//      per entry: every entry is one operation whose inputs are final, and
//      a host-built program runs the operations of one dependency level side
//      by side on the cell's lanes;
//   3. the strict lower part L_s and the row-scaled strict upper part
//      D^-1 U_s (D = diag(U)) are taken into registers, each in a sliced-ELL
//      schedule of its own (rows dealt by their own lengths, so the short
//      triangle rows are not padded to A's row lengths), together with D^-1.
// Each application of M^-1 to q solves L y = q and then U z = y by s Jacobi
// sweeps each: y <- q, then s times y <- q - L_s y; z <- D^-1 y, then s times
// z <- D^-1 y - (D^-1 U_s) z.  That is the Neumann series of each triangle
// truncated after s terms, a fixed linear operator, and exact once s reaches
// the triangle's dependency depth.  All three schedules gather from the
// slot's one operand block, through which vectors also move between the
// three row dealings.  Outside the preconditioner the iteration is the one
// of the FP64 kernel (bcs_fp64.h): the same stopping tests, true-residual
// confirmation, residual replacement, breakdown restarts and initial guess.
#pragma once

#include "bcs_device.h"

namespace bcs {
namespace dev {

// The factorisation program of one pattern and lane count: NSTEP steps, step
// st with W_st terms.  Words of step st (from offset(st)): LANES head words
// (target position | divisor position << 16), then W_st x LANES term words
// (position of l_ik | position of u_kj << 16), lane-minor.  Positions index
// the slot's factor block (16 bits; past the NNZ values: kIluZero,
// kIluUnit, kIluJunk).
template <int NNZ_, int... W>
struct FactProg {
  static constexpr int NNZ = NNZ_;
  static constexpr int NSTEP = sizeof...(W);
  static constexpr int width(int st) {
    constexpr int w[] = {W..., 0};
    return w[st];
  }
  static constexpr int offset(int st, int lanes) {
    constexpr int w[] = {W..., 0};
    int o = 0;
    for (int q = 0; q < st; ++q) o += (1 + w[q]) * lanes;
    return o;
  }
};

// Run steps ST.. of the program on the factor block F: each lane takes one
// operation per step, acc = F[target] - sum_q F[l_q] F[u_q] (terms in
// increasing k), F[target] = acc / F[divisor] (the divisor of an upper-part
// operation is the constant 1).  A padding operation reads 0 * 0 terms and
// rewrites kIluJunk.
template <class FP, int LANES, int ST = 0>
__device__ __forceinline__ void ilu_factor(double* F, const uint32_t* prog, int gl) {
  if constexpr (ST < FP::NSTEP) {
    constexpr int W = FP::width(ST);
    constexpr int OFF = FP::offset(ST, LANES);
    const uint32_t head = prog[OFF + gl];
    uint32_t tw[W > 0 ? W : 1];
#pragma unroll
    for (int q = 0; q < W; ++q) tw[q] = prog[OFF + (1 + q) * LANES + gl];
    double acc = F[head & 0xffffu];
#pragma unroll
    for (int q = 0; q < W; ++q) acc = __builtin_fma(-F[tw[q] & 0xffffu], F[tw[q] >> 16], acc);
    acc = acc / F[head >> 16];
    F[head & 0xffffu] = acc;
    wave_sync();
    ilu_factor<FP, LANES, ST + 1>(F, prog, gl);
  }
}

}  // namespace dev

// Owned rows of a schedule (a padding row, -1 or the spanning lane's second
// slot, stages into the spare element n).
template <int RPL, int LANES>
__device__ __forceinline__ void owned_rows(const DevSchedule& d, int n, int gl, int (&rows)[RPL]) {
#pragma unroll
  for (int j = 0; j < RPL; ++j) {
    const int rj = d.row[j * LANES + gl];
    rows[j] = rj >= 0 ? rj : n;
  }
}

// SA: schedule of A; SL / SU: schedules of L_s and U_s; FP: the
// factorisation program.
template <class SA, class SL, class SU, class FP>
__device__ __forceinline__ void ilu_body(const KParams& P) {
  using namespace dev;
  constexpr int LANES = SA::LANES;
  static_assert(SL::LANES == LANES && SU::LANES == LANES, "one lane count for all schedules");
  static_assert((SL::FLAGS & kSchedDiag) == 0 && (SU::FLAGS & kSchedDiag) == 0,
                "the strict triangles hold no diagonal");
  constexpr int RA = SA::RPL, RL = SL::RPL, RU = SU::RPL;
  constexpr int KA = SA::KMAX, KL = SL::KMAX, KU = SU::KMAX;
  constexpr int NNZ = FP::NNZ;
  constexpr int ZERO = NNZ + kIluZero, UNIT = NNZ + kIluUnit, JUNK = NNZ + kIluJunk;
  extern __shared__ double lds[];

  // The workgroup's copy of the tables: value positions of the three
  // schedules, each row's diagonal position (row n, the padding row: UNIT),
  // then the factorisation program.
  uint16_t* tab = (uint16_t*)(lds + P.tbase);
  const int ntab = (KA + KL + KU) * LANES + P.n + 1;
  for (int i = threadIdx.x; i < ntab; i += kWgThreads) tab[i] = P.ilu_tab[i];
  uint32_t* prog = (uint32_t*)(tab + ((ntab + 1) & ~1));
  for (int i = threadIdx.x; i < P.fprog_words; i += kWgThreads) prog[i] = P.fprog[i];
  __syncthreads();
  const uint16_t* entA = tab;
  const uint16_t* entL = entA + KA * LANES;
  const uint16_t* entU = entL + KL * LANES;
  const uint16_t* dpos = entU + KU * LANES;

  const SA sa(P.sched);
  const SL sl(P.schedL);
  const SU su(P.schedU);
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int gl = lane & (LANES - 1);
  const int grp = lane / LANES;
  // the slot's block: the factor block while a cell is staged, afterwards
  // the operand block X (n values and the zero spare element n)
  double* F = lds + (wv * (64 / LANES) + grp) * P.fs;
  double* X = F;
  const int n = P.n;

  uint32_t adA[SA::NW], adL[SL::NW], adU[SU::NW];
  build_addr<SA::PACK, KA, LANES>(adA, P.sched.col, lds_addr(X), gl);
  build_addr<SL::PACK, KL, LANES>(adL, P.schedL.col, lds_addr(X), gl);
  build_addr<SU::PACK, KU, LANES>(adU, P.schedU.col, lds_addr(X), gl);
  int rowsA[RA], rowsL[RL], rowsU[RU];
  owned_rows<RA, LANES>(P.sched, n, gl, rowsA);
  owned_rows<RL, LANES>(P.schedL, n, gl, rowsL);
  owned_rows<RU, LANES>(P.schedU, n, gl, rowsU);
  // 1 on a lane whose slots 0 and 1 hold one long row, per schedule
  double spanA = 0, spanL = 0, spanU = 0;
  if constexpr (SA::SPAN) spanA = (P.sched.row[LANES + gl] == kRowSpan) ? 1.0 : 0.0;
  if constexpr (SL::SPAN) spanL = (P.schedL.row[LANES + gl] == kRowSpan) ? 1.0 : 0.0;
  if constexpr (SU::SPAN) spanU = (P.schedU.row[LANES + gl] == kRowSpan) ? 1.0 : 0.0;

  double a[KA], aL[KL], aU[KU];  // A, L_s, D^-1 U_s on this lane's schedule steps
  double dgv[RA];                // A's diagonal in the owned rows (1 in padding rows)
  double uinv[RU];               // D^-1 in the U dealing's owned rows (1 in padding rows)
  double xv[RA], r[RA], rh[RA], p[RA], v[RA], t[RA], bb[RA], ph[RA], sh[RA];
  const double none[RL] = {};
  const double noneU[RU] = {};
  double bn = 0, tol2 = 0, rho = 0, rho_prev = 1, alpha = 1, omega = 1;
  bool warm = false;
  int it = 0, restarts_left = 0;
  bool active = false, dead = false;
  int64_t cell = 0;
  int32_t held[kClaimGroup - 1];
#pragma unroll
  for (int q = 0; q < kClaimGroup - 1; ++q) held[q] = -1;
  held[0] = initial_held(P.queue, P.qfirst, P.ncells, wv, grp, 64 / LANES);

  auto finish = [&](int st, double res) {
    if (warm) {
      const double* x0c = P.x0 + cell * n;
#pragma unroll
      for (int j = 0; j < RA; ++j)
        if (rowsA[j] < n) xv[j] = x0c[rowsA[j]] + xv[j];
    }
#pragma unroll
    for (int j = 0; j < RA; ++j)
      if (rowsA[j] < n) P.x[cell * n + rowsA[j]] = xv[j];
    if (gl == 0) {
      P.iters[cell] = it;
      P.resid[cell] = res;
      P.status[cell] = st;
      if (P.refinements) P.refinements[cell] = 0;
#ifdef BCS_COUNT_VISITS
      if (P.visits) atomicAdd(P.visits + cell, 1);  // debug: outputs written per cell
#endif
    }
    active = false;
  };

  auto restart = [&]() {
#pragma unroll
    for (int j = 0; j < RA; ++j) {
      rh[j] = r[j];
      p[j] = 0;
      v[j] = 0;
    }
    rho_prev = alpha = omega = 1;
  };

  // out = M^-1 q (A dealing), left in X as well (every row, 0 in the spare
  // element) for the SpMV that follows.
  auto minv = [&](const double (&q)[RA], double (&out)[RA]) {
#pragma unroll
    for (int j = 0; j < RA; ++j) X[rowsA[j]] = q[j];
    wave_sync();
    double qL[RL], y[RL], acc[RL];
#pragma unroll
    for (int j = 0; j < RL; ++j) qL[j] = X[rowsL[j]];
    // first sweep from y = q, which X already holds
    sl.template spmv<double, false>(aL, adL, X, nullptr, gl, rowsL, qL, acc, none, spanL);
#pragma unroll
    for (int j = 0; j < RL; ++j) y[j] = qL[j] - acc[j];
    for (int m = 1; m < P.sweeps; ++m) {
      sl.spmv(aL, adL, X, nullptr, gl, rowsL, y, acc, none, spanL);
#pragma unroll
      for (int j = 0; j < RL; ++j) y[j] = qL[j] - acc[j];
    }
#pragma unroll
    for (int j = 0; j < RL; ++j) X[rowsL[j]] = y[j];
    wave_sync();
    double yh[RU], z[RU], accU[RU];
#pragma unroll
    for (int j = 0; j < RU; ++j) {
      yh[j] = uinv[j] * X[rowsU[j]];
      z[j] = yh[j];
    }
    for (int m = 0; m < P.sweeps; ++m) {
      su.spmv(aU, adU, X, nullptr, gl, rowsU, z, accU, noneU, spanU);
#pragma unroll
      for (int j = 0; j < RU; ++j) z[j] = yh[j] - accU[j];
    }
#pragma unroll
    for (int j = 0; j < RU; ++j) X[rowsU[j]] = z[j];
    wave_sync();
#pragma unroll
    for (int j = 0; j < RA; ++j) out[j] = X[rowsA[j]];
  };

  for (;;) {
    if (!active && !dead) {
      if (!claim_cell(P.queue, P.order, P.ncells, grp * LANES, gl == 0, cell, held, wv, grp, 64 / LANES)) {
        dead = true;
      } else {
        if constexpr (LANES == 64) {
          // one cell per wave: keep its index in scalar registers
          const uint64_t u = (uint64_t)cell;
          cell = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(u >> 32)) << 32) |
                           (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u));
        }
        // 1. A into the factor block: -(gamma J) at every position, then
        //    1 + that on the diagonal (which rounds as 1 - gamma J does)
        const double* vals = P.values + cell * NNZ;
        const double g = (P.kind == kJGamma) ? P.gamma[cell * P.gamma_stride] : 0.0;
        constexpr int NV = (NNZ + LANES - 1) / LANES;
#pragma unroll
        for (int m = 0; m < NV; ++m) {
          const int k = m * LANES + gl;
          if (k < NNZ) F[k] = (P.kind == kJGamma) ? -(g * vals[k]) : vals[k];
        }
        if (gl == 0) {
          F[ZERO] = 0.0;
          F[UNIT] = 1.0;
          F[JUNK] = 0.0;
        }
        wave_sync();
        if (P.kind == kJGamma) {
#pragma unroll
          for (int j = 0; j < RA; ++j)
            if (rowsA[j] < n) {
              const int d = dpos[rowsA[j]];
              F[d] = 1.0 + F[d];
            }
          wave_sync();
        }
        // 2. A's values and diagonal into registers
#pragma unroll
        for (int s = 0; s < KA; ++s) a[s] = F[entA[s * LANES + gl]];
#pragma unroll
        for (int j = 0; j < RA; ++j) dgv[j] = F[dpos[rowsA[j]]];
        // 3. the incomplete factors in place
        ilu_factor<FP, LANES>(F, prog, gl);
        // 4. L_s, D^-1 and D^-1 U_s into registers (a spanning lane's slot 1
        //    belongs to its slot-0 row)
#pragma unroll
        for (int s = 0; s < KL; ++s) aL[s] = F[entL[s * LANES + gl]];
#pragma unroll
        for (int j = 0; j < RU; ++j) uinv[j] = 1.0 / F[dpos[rowsU[j]]];
        if constexpr (SU::SPAN) uinv[1] = spanU != 0.0 ? uinv[0] : uinv[1];
#pragma unroll
        for (int s = 0; s < KU; ++s) aU[s] = F[entU[s * LANES + gl]] * uinv[SU::slot_of(s)];
        wave_sync();
        if (gl == 0) X[n] = 0.0;  // the operand block's spare element (X overlays F)
        wave_sync();

        const double* bc = P.b + cell * n;
#pragma unroll
        for (int j = 0; j < RA; ++j) {
          const bool real = rowsA[j] < n;
          const double bj = bc[real ? rowsA[j] : 0];
          bb[j] = real ? bj : 0.0;
          r[j] = bb[j];
          xv[j] = 0;
        }
        // Initial guess: iterate on the correction from r0 = b - A x0 (kept
        // in t), with relative residuals still relative to ||b||.
        const bool use_x0 = P.x0 != nullptr;
        if (use_x0) {
          const double* x0c = P.x0 + cell * n;
          double x0v[RA];
#pragma unroll
          for (int j = 0; j < RA; ++j) x0v[j] = (rowsA[j] < n) ? x0c[rowsA[j]] : 0.0;
          sa.spmv(a, adA, X, nullptr, gl, rowsA, x0v, t, dgv, spanA);
#pragma unroll
          for (int j = 0; j < RA; ++j) t[j] = bb[j] - t[j];
        }
        const double bn2 = gsum<LANES>(ldot<RA>(r, r));
        bn = __builtin_sqrt(bn2);
        tol2 = (P.rtol * bn) * (P.rtol * bn);
        double rr2 = bn2;
        warm = use_x0 && finite(bn) && bn != 0.0;
        if (warm) {
#pragma unroll
          for (int j = 0; j < RA; ++j) bb[j] = r[j] = t[j];
          rr2 = gsum<LANES>(ldot<RA>(r, r));
        }
        it = 0;
        restarts_left = P.brs;
        restart();
        rho = rr2;
        active = true;
        if (!finite(bn)) {
          finish(kNonfinite, __builtin_nan(""));
        } else if (bn == 0.0) {
          finish(kConverged, 0.0);
        } else if (rr2 <= tol2) {
          finish(kConverged, __builtin_sqrt(rr2) / bn);
        }
      }
    }
    if (__ballot(!dead) == 0ull) break;
    if (!active) continue;

    // ---- one preconditioned BiCGStab iteration of this slot's cell ----
    ++it;
    int ended = -1;
    if (!finite(rho)) {
      ended = kNonfinite;
    } else if (rho == 0.0) {
      ended = kBreakdown;
    } else {
      const double beta = qdiv(rho * alpha, rho_prev * omega);
#pragma unroll
      for (int j = 0; j < RA; ++j) p[j] = r[j] + beta * (p[j] - omega * v[j]);
      minv(p, ph);
      sa.template spmv<double, false>(a, adA, X, nullptr, gl, rowsA, ph, v, dgv, spanA);
      const double sigma = gsum<LANES>(ldot<RA>(rh, v));
      if (!finite(sigma)) {
        ended = kNonfinite;
      } else if (sigma == 0.0) {
        ended = kBreakdown;
      } else {
        alpha = qdiv(rho, sigma);
#pragma unroll
        for (int j = 0; j < RA; ++j) r[j] = r[j] - alpha * v[j];  // r now holds s
        // t = A M^-1 s before the half-step test, so that ||s||^2, (t, s)
        // and (t, t) are reduced together
        minv(r, sh);
        sa.template spmv<double, false>(a, adA, X, nullptr, gl, rowsA, sh, t, dgv, spanA);
        double red3[3] = {ldot<RA>(r, r), ldot<RA>(t, t), ldot<RA>(t, r)};
        gsum_n<LANES>(red3);
        const double sn2 = red3[0], tt = red3[1], ts = red3[2];
        if (!finite(sn2)) {
          ended = kNonfinite;
        } else if (sn2 <= tol2) {
#pragma unroll
          for (int j = 0; j < RA; ++j) xv[j] = xv[j] + alpha * ph[j];
          ended = kConverged;
        } else if (!finite(tt)) {
          ended = kNonfinite;
        } else if (tt == 0.0) {
          ended = kBreakdown;
        } else {
          omega = qdiv(ts, tt);
#pragma unroll
          for (int j = 0; j < RA; ++j) {
            xv[j] = xv[j] + alpha * ph[j] + omega * sh[j];
            r[j] = r[j] - omega * t[j];
          }
          // ||r||^2 = ||s||^2 - omega (t, s) for omega = (t, s) / (t, t)
          const double rn2 = sn2 - omega * ts;
          const double rho_next = gsum<LANES>(ldot<RA>(rh, r));
          if (!finite(rn2)) {
            ended = kNonfinite;
          } else if (rn2 <= tol2) {
            ended = kConverged;
          } else if (omega == 0.0) {
            ended = kBreakdown;
          } else {
            rho_prev = rho;
            rho = rho_next;
          }
        }
      }
    }
    if (ended < 0 && it >= P.maxit) ended = kMaxit;
    if (ended >= 0) {
      sa.spmv(a, adA, X, nullptr, gl, rowsA, xv, t, dgv, spanA);
#pragma unroll
      for (int j = 0; j < RA; ++j) t[j] = bb[j] - t[j];
      const double tt2 = gsum<LANES>(ldot<RA>(t, t));
      const double res = __builtin_sqrt(tt2) / bn;
      if (ended == kNonfinite || !finite(res)) {
        finish(kNonfinite, res);
      } else if (res <= P.rtol) {
        finish(kConverged, res);
      } else if (it < P.maxit && ((ended == kConverged && P.rr) || (ended == kBreakdown && restarts_left > 0))) {
        if (ended == kBreakdown) --restarts_left;
#pragma unroll
        for (int j = 0; j < RA; ++j) r[j] = t[j];
        restart();
        rho = tt2;
      } else {
        finish(ended == kBreakdown ? kBreakdown : kMaxit, res);
      }
    }
  }
}

}  // namespace bcs
