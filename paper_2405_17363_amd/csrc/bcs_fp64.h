// FP64 batched Block-cells BiCGStab kernel (forward solve and adjoint solve).
//
// One launch solves every cell: a persistent grid whose cell slots (LANES
// lanes each) pull cell indices from a device work queue, iterate that cell's
// BiCGStab to completion without any inter-workgroup communication or host
// round trip (the Block-cells arrangement, Section 3.1), write the cell's
// outputs and pull the next cell.  Slots of one wave advance independently:
// a slot whose cell has converged refills while its neighbours iterate.
//
// Per iteration (right preconditioning M = diag(A) when enabled):
//   rho = (rhat, r);  p = r + beta (p - omega v);  v = A M^-1 p;  sigma = (rhat, v)
//   alpha = rho / sigma;  s = r - alpha v;  stop if ||s|| <= rtol ||b||
//   t = A M^-1 s;  omega = (t, s) / (t, t);  x += alpha M^-1 p + omega M^-1 s
//   r = s - omega t;  stop if ||r|| <= rtol ||b||
// (||r||^2 = ||s||^2 - omega (t, s), an identity, so that the last reduction
// of the iteration carries only (rhat, r)).  Then the true residual
// ||b - A x|| confirms convergence; a cell whose true residual misses rtol
// restarts from it (residual replacement) while iterations remain, and an
// exact breakdown restarts a bounded number of times.  With an initial guess
// x0 the loop solves for the correction x - x0.  The adjoint mode runs the
// same loop on A^T (a transposed schedule over the same per-cell values) with
// g as right-hand side and then writes dL/dA_ij = -lambda_i x_j (or its chain
// rule to J and gamma for A = I - gamma J).
#pragma once

#include "bcs_device.h"

namespace bcs {

// One mechanism's persistent solve loop: this wave's cell slots claim cells
// from the work queue P.queue until it is exhausted.  `lds` is the
// workgroup's LDS base, wv the wave's index in the workgroup, ent_lds and
// diag_lds the LDS copies of the schedule's value positions and of the
// diagonal's position in every row.
// ADJ: -1 = forward or adjoint chosen by P.adjoint at run time (the
// precompiled generic kernels), 0 = forward only, 1 = adjoint only (kernels
// compiled per pattern, which then carry no code for the other mode).
// GRP: Block-cells (N) (Section 3): the wave's 64 / LANES cells, consecutive
// cells claimed together, are one system (the block-diagonal matrix of its
// cells): every inner product, scalar and stopping test spans the wave.  A
// slot past the last cell is padding with all-zero data.  Each cell reports
// the run's iterations, its own true residual and CONVERGED only if that
// residual is within rtol.
// MT (a dev::MechTerms): the cell's J is assembled while it is staged, from
// its concentrations and the kernel's J term program (P.y, P.kr, P.mtab), in
// the order and rounding of the assembly kernel, instead of being read from
// P.values.
template <class S, int ADJ = -1, bool GRP = false, class MT = dev::NoMechTerms>
__device__ __forceinline__ void fp64_run(const KParams& P, double* lds, int wv, const int32_t* ent_lds,
                                         const int32_t* diag_lds) {
  using namespace dev;
  static_assert(!GRP || ADJ == 0, "shared scalars: forward solves only");
  constexpr bool MECH = MT::kOn;
  static_assert(!MECH || MT::kP == S::KMAX + S::RPL, "J term program: one entry per schedule step and row");
  const bool adjoint = ADJ < 0 ? (P.adjoint != 0) : (ADJ == 1);
  constexpr int LANES = S::LANES, RPL = S::RPL, KMAX = S::KMAX;
  constexpr int RL = GRP ? 64 : LANES;  // lanes an inner product spans
  const S sch(P.sched);
  constexpr int NW = S::NW, PACK = S::PACK;
  const int lane = threadIdx.x & 63;
  const int gl = lane & (LANES - 1);
  const int grp = lane / LANES;
  double* xb = lds + wv * P.wxs + grp * P.xs;                    // SpMV operand (n + spare)
  double* yb = lds + P.bbase + wv * P.wbs + grp * P.bs + P.yoff;  // SpMV result, slot-major RPL x LANES

  const int n = P.n, nnz = P.nnz;

  // This lane's LDS gather addresses (the schedule is shared by every cell
  // of the plan and padded to exactly KMAX steps).
  uint32_t ad[NW];
  build_addr<PACK, KMAX, LANES>(ad, P.sched.col, lds_addr(xb), gl);
  // Owned rows; a padding row (-1) stages into the spare LDS element n.
  // Padding rows only ever store 0 there, and padding steps of the schedule
  // gather it, so it starts at 0 and a padding step adds value * 0.
  if (gl == 0) xb[n] = 0.0;
  if constexpr (MECH) {
    if (gl == 0) xb[n + 1] = 1.0;  // y factor of the first-order J terms
  }
  wave_sync();
  int rows[RPL];
#pragma unroll
  for (int j = 0; j < RPL; ++j) {
    const int rj = P.sched.row[j * LANES + gl];
    rows[j] = rj >= 0 ? rj : n;
  }

  double a[KMAX];
  // Krylov state of this lane's rows.  With Jacobi the matrix is staged
  // column-scaled (Ahat = A D^-1, right preconditioning), so the iterate
  // holds xhat = D x and x = D^-1 xhat is formed when the cell finishes.
  // r, p, v and t, which every step of the iteration reads, stay in
  // registers.  Kernels built with kSchedLean keep the iterate and the
  // shadow residual (read or updated once or twice per iteration) and b and
  // diag(A)^-1 (read when a cell ends or restarts) in the slot's state block
  // in LDS instead, each lane's own words (no other lane reads them, so they
  // need no synchronisation); with packed addresses that brings the n = 80
  // kernel at 32 lanes within the registers of three waves per SIMD.
  double r[RPL], p[RPL], v[RPL], t[RPL];
  constexpr bool LEAN = (S::FLAGS & kSchedLean) != 0;
  constexpr int RR = LEAN ? 1 : RPL;
  double xv_r[RR], rh_r[RR], bb_r[RR], dinv_r[RR];  // the same vectors in registers (not LEAN)
  double* const sv = lds + P.bbase + wv * P.wbs + grp * P.bs + gl;  // LEAN: [kSlotVecs][RPL][LANES]
  auto XV = [&](int j) -> double& {
    if constexpr (LEAN) return sv[(kSlotX * RPL + j) * LANES]; else return xv_r[j];
  };
  auto RH = [&](int j) -> double& {
    if constexpr (LEAN) return sv[(kSlotRhat * RPL + j) * LANES]; else return rh_r[j];
  };
  auto BB = [&](int j) -> double& {
    if constexpr (LEAN) return sv[(kSlotB * RPL + j) * LANES]; else return bb_r[j];
  };
  auto DINV = [&](int j) -> double& {
    if constexpr (LEAN) return sv[(kSlotDinv * RPL + j) * LANES]; else return dinv_r[j];
  };
  auto load_vec = [&](auto& ref, double (&out)[RPL]) {
#pragma unroll
    for (int j = 0; j < RPL; ++j) out[j] = ref(j);
  };
  // Schedules without diagonal entries: the staged (column-scaled) diagonal
  // value of each owned row, 0 for padding rows.
  double dgv[RPL];
#pragma unroll
  for (int j = 0; j < RPL; ++j) dgv[j] = 0;
  // 1 on a lane whose slots 0 and 1 hold one long row
  double span = 0;
  if constexpr (S::FLAGS & kSchedSpan) span = (P.sched.row[LANES + gl] == kRowSpan) ? 1.0 : 0.0;
  double bn = 0, tol2 = 0, rho = 0, rho_prev = 1, alpha = 1, omega = 1;
  double gam = 0;     // the cell's gamma (adjoint chain rule)
  bool warm = false;  // the cell starts from the caller's x0
  int it = 0, restarts_left = 0;
  bool active = false, dead = false;
  int64_t cell = 0;
  bool pad = false;  // GRP: a slot past the last cell
  double bnc = 0;    // GRP: ||b|| of this slot's own cell
  int32_t held[kClaimGroup - 1];  // cells claimed and not yet started
#pragma unroll
  for (int q = 0; q < kClaimGroup - 1; ++q) held[q] = -1;
  held[0] = initial_held(P.queue, P.qfirst, P.ncells, wv, grp, 64 / LANES);

  // Write the cell's outputs and free the slot.
  auto finish = [&](int st, double res) {
    if (GRP && pad) {
      active = false;
      return;
    }
    double xv[RPL];
    load_vec(XV, xv);
    if (P.precond) {
#pragma unroll
      for (int j = 0; j < RPL; ++j) xv[j] = DINV(j) * xv[j];
    }
    if (warm) {
      const double* x0c = P.x0 + cell * n;
#pragma unroll
      for (int j = 0; j < RPL; ++j)
        if (rows[j] < n) xv[j] = x0c[rows[j]] + xv[j];
    }
    if (adjoint) {
      // lambda through the slot's LDS block, so every lane reaches every row
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        xb[rows[j]] = xv[j];
      }
      wave_sync();
      // and the forward solution x through the slot's SpMV result block (free
      // once the last SpMV is done; RPL x LANES >= n words)
      {
        const double* xc = P.xin + cell * n;
        double xl[RPL];
#pragma unroll
        for (int j = 0; j < RPL; ++j) xl[j] = gl + j * LANES < n ? xc[gl + j * LANES] : 0.0;
#pragma unroll
        for (int j = 0; j < RPL; ++j)
          if (gl + j * LANES < n) yb[gl + j * LANES] = xl[j];
      }
      wave_sync();
      // entry k = (i, j): lambda_i x_j; dL/dA_k = -lambda_i x_j, and in J mode
      // dL/dJ_k = gamma lambda_i x_j and dL/dgamma = sum_k J_k lambda_i x_j.
      // Consecutive lanes write consecutive positions; (i, j) of each position
      // come from the workgroup's LDS copy.
      const bool to_j = P.grad_kind == 1 && P.kind == kJGamma;
      const double* vals = P.values + cell * nnz;
      const uint32_t* coo = (const uint32_t*)(lds + P.coobase);
      double gpart = 0;
#pragma unroll 4
      for (int k = gl; k < nnz; k += LANES) {
        const uint32_t w = coo[k];
        const double lx = xb[w & 0xffffu] * yb[w >> 16];
        P.grad_vals[cell * nnz + k] = to_j ? gam * lx : -lx;
        if (P.grad_gamma) gpart = __builtin_fma(vals[k], lx, gpart);
      }
      if (P.grad_gamma) {
        const double tot = gsum<LANES>(gpart);
        if (gl == 0) P.grad_gamma[cell] = tot;
      }
      wave_sync();
    }
#pragma unroll
    for (int j = 0; j < RPL; ++j)
      if (rows[j] < n) P.x[cell * n + rows[j]] = xv[j];
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

  // Restart the recurrences from the current r.
  auto restart = [&]() {
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      RH(j) = r[j];
      p[j] = 0;
      v[j] = 0;
    }
    rho_prev = alpha = omega = 1;
  };

  for (;;) {
    if (!active && !dead) {
      bool claimed;
      if constexpr (GRP) {
        // the wave's run of consecutive cells
        unsigned long long c = 0;
        if (lane == 0) c = atomicAdd(P.queue, (unsigned long long)(64 / LANES));
        c = __shfl(c, 0, 64);
        claimed = c < (unsigned long long)P.ncells;
        cell = (int64_t)c + grp;
        pad = cell >= P.ncells;
        if (pad) cell = 0;  // loads stay in bounds; the data is zeroed below
      } else {
        claimed = claim_cell(P.queue, P.order, P.ncells, grp * LANES, gl == 0, cell, held, wv, grp, 64 / LANES);
        if constexpr (LANES == 64) {
          // one cell per wave: keep its index in scalar registers
          const uint64_t u = (uint64_t)cell;
          cell = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(u >> 32)) << 32) |
                           (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u));
        }
      }
      if (!claimed) {
        dead = true;
      } else {
        // Stage the cell: A = I - gamma J (or A) into registers, b, and the
        // Jacobi column scaling.  Value positions come from the LDS copy of
        // the schedule, so every global load of the cell is independent and
        // they all issue back to back (one memory latency per refill).
        const double* vals = P.values + cell * nnz;
        const double g = (P.kind == kJGamma) ? P.gamma[cell * P.gamma_stride] : 0.0;
        gam = g;
        const double* bc = P.b + cell * n;
        double dv[RPL];
        double bl[RPL];  // b of the owned rows, loaded early when J is assembled here
        if constexpr (MECH) {
          // J of this cell at the schedule's positions and at its rows'
          // diagonals: the concentrations go through the operand block (rows
          // 0 .. n-1; the spare element n keeps its zero), then every lane
          // runs its J term program, each position's terms in reaction order
          // (padding terms have no reaction and add nothing)
          const double* yc = P.y + cell * n;
          {
            // b and y: all loads in flight at once (RPL x LANES >= n)
#pragma unroll
            for (int j = 0; j < RPL; ++j) bl[j] = bc[rows[j] < n ? rows[j] : 0];
            double yl[RPL];
#pragma unroll
            for (int j = 0; j < RPL; ++j) yl[j] = gl + j * LANES < n ? yc[gl + j * LANES] : 0.0;
#pragma unroll
            for (int j = 0; j < RPL; ++j)
              if (gl + j * LANES < n) xb[gl + j * LANES] = yl[j];
          }
          wave_sync();
          const uint2* prog = (const uint2*)(lds + P.mtbase + P.mr + 2) + gl;
          const uint32_t xaddr = lds_addr(xb);
          // Rate constants from LDS (shared; after them a zero, which padding
          // terms read, and a one) or from the cell's row in memory: two
          // copies of the program, each with its address space.  A term takes
          // no branch: the y factor of a first-order term is the 1 at
          // xb[n + 1], the factor 2 an exact ldexp by 1 or 0.  k y rounds once
          // and S d is exact in the FMA, as in the assembly kernel, so the
          // sums are bitwise its sums.  First every lane evaluates position 0
          // and the slot's first lane keeps it at xb[n + 2]; a padding step's
          // single term then reads it there (1 x J0, S = 1: exactly J0).
          auto jprog = [&](auto mode) {
            constexpr bool SHARED = decltype(mode)::value == 0;
            const double* kc = P.kr + cell * P.k_stride;
            const uint32_t kb = (uint32_t)P.mtbase * 8u;
            auto term = [&](uint2 w, double kv, double yv, double acc) {
              const double sf = __builtin_bit_cast(double, (uint64_t)w.y << 32);
              double k = kv;
              if constexpr (!SHARED) {
                const uint32_t r = ((w.x & 0xfff8u) - kb) >> 3;
                k = r < (uint32_t)P.mr ? k : (r == (uint32_t)P.mr + 1 ? 1.0 : 0.0);
              }
              return fmat(sf, __builtin_amdgcn_ldexp(k * yv, (int)(w.x & 1u)), acc);
            };
            auto kload = [&](uint2 w) -> double {
              const uint32_t ka = w.x & 0xfff8u;
              if constexpr (SHARED) {
                return lds_load<double>(ka);
              } else {
                const uint32_t r = (ka - kb) >> 3;
                return kc[r < (uint32_t)P.mr ? r : 0];  // the constants after them are taken in term()
              }
            };
            {
              constexpr int J0 = MT::kJ0;
              double j0 = 0.0;
              if constexpr (J0 > 0) {
                uint2 w[J0];
                double kv[J0], yv[J0];
#pragma unroll
                for (int t = 0; t < J0; ++t) w[t] = prog[t * LANES];
#pragma unroll
                for (int t = 0; t < J0; ++t) {
                  kv[t] = kload(w[t]);
                  yv[t] = lds_load<double>(xaddr + (w[t].x >> 16));
                }
#pragma unroll
                for (int t = 0; t < J0; ++t) j0 = term(w[t], kv[t], yv[t], j0);
              }
              if (gl == 0) xb[n + 2] = j0;
              wave_sync();
            }
            const uint2* mprog = prog + MT::kJ0 * LANES;
#pragma unroll
            for (int q = 0; q < KMAX; ++q) a[q] = 0.0;
#pragma unroll
            for (int j = 0; j < RPL; ++j) dv[j] = 0.0;
            // kJTermChunk terms at a time: their operands, then their
            // arithmetic, so that the loads of a chunk are in flight
            // together; the next chunk's program words are read meanwhile
            constexpr int U = MT::total();
            uint2 wn[kJTermChunk];
#pragma unroll
            for (int g = 0; g < kJTermChunk; ++g)
              if (g < U) wn[g] = mprog[g * LANES];
            for_pos<0, (U + kJTermChunk - 1) / kJTermChunk>([&](auto chunk) {
              constexpr int u0 = decltype(chunk)::value * kJTermChunk;
              constexpr int G = U - u0 < kJTermChunk ? U - u0 : kJTermChunk;
              constexpr int u1 = u0 + kJTermChunk;
              uint2 w[G];
              double kv[G], yv[G];
#pragma unroll
              for (int g = 0; g < G; ++g) w[g] = wn[g];
#pragma unroll
              for (int g = 0; g < G; ++g) {
                kv[g] = kload(w[g]);
                yv[g] = lds_load<double>(xaddr + (w[g].x >> 16));
              }
#pragma unroll
              for (int g = 0; g < kJTermChunk; ++g)
                if (u1 + g < U) wn[g] = mprog[(u1 + g) * LANES];
              for_pos<0, G>([&](auto gg) {
                constexpr int g = decltype(gg)::value;
                constexpr int q = MT::pos_of(u0 + g);
                if constexpr (q < KMAX)
                  a[q] = term(w[g], kv[g], yv[g], a[q]);
                else
                  dv[q - KMAX] = term(w[g], kv[g], yv[g], dv[q - KMAX]);
              });
            });
          };
          if (P.k_stride)
            jprog(Pos<1>{});
          else
            jprog(Pos<0>{});
          wave_sync();
        } else {
#pragma unroll
          for (int s = 0; s < KMAX; ++s) a[s] = vals[ent_lds[s * LANES + gl] & kEntPosMask];
#pragma unroll
          for (int j = 0; j < RPL; ++j) dv[j] = vals[diag_lds[rows[j] < n ? rows[j] : 0]];
        }
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
          const bool real = rows[j] < n;
          const double bj = MECH ? bl[j] : bc[real ? rows[j] : 0];
          r[j] = real ? bj : 0.0;
          BB(j) = r[j];
          XV(j) = 0;
        }
        // A = I - gamma J on the schedule's entries (a padding step keeps the
        // finite value it loaded: it multiplies the zero spare element)
        if constexpr ((S::FLAGS & kSchedDiag) != 0) {
          // no diagonal entries in the schedule
#pragma unroll
          for (int s = 0; s < KMAX; ++s) a[s] = (P.kind == kJGamma) ? -g * a[s] : a[s];
        } else {
          asm volatile("" ::: "memory");  // re-read the flags below instead of keeping them live
#pragma unroll
          for (int s = 0; s < KMAX; ++s) {
            const int32_t e = ent_lds[s * LANES + gl];
            a[s] = (P.kind == kJGamma) ? (((e & kEntDiag) ? 1.0 : 0.0) - g * a[s]) : a[s];
          }
        }
        if constexpr ((S::FLAGS & kSchedDiag) != 0) {
#pragma unroll
          for (int j = 0; j < RPL; ++j) {
            const double d = (P.kind == kJGamma) ? 1.0 - g * dv[j] : dv[j];
            dgv[j] = (rows[j] < n) ? d : 0.0;
          }
        }
        // Initial guess x0: the iteration runs on the correction e = x - x0,
        // A e = r0 = b - A x0 from e = 0, with r0 in place of b in the
        // true-residual checks (relative residuals stay relative to ||b||).
        // r0 is formed here with the unscaled matrix and kept in t.
        const bool use_x0 = !GRP && P.x0 != nullptr;
        if (use_x0) {
          const double* x0c = P.x0 + cell * n;
          double x0v[RPL];
#pragma unroll
          for (int j = 0; j < RPL; ++j) x0v[j] = (rows[j] < n) ? x0c[rows[j]] : 0.0;
          sch.spmv(a, ad, xb, yb, gl, rows, x0v, t, dgv, span);
#pragma unroll
          for (int j = 0; j < RPL; ++j) t[j] = r[j] - t[j];
        }
        if (P.precond) {
          // column scaling by diag(A)^-1, gathered through the LDS slice
#pragma unroll
          for (int j = 0; j < RPL; ++j) {
            const double d = (P.kind == kJGamma) ? 1.0 - g * dv[j] : dv[j];
            const double di = (rows[j] < n) ? 1.0 / d : 0.0;
            DINV(j) = di;
            xb[rows[j]] = di;
            if constexpr ((S::FLAGS & kSchedDiag) != 0) dgv[j] *= di;
          }
          wave_sync();
          uint32_t ado[NW];
          opaque_copy<NW>(ad, ado);
#pragma unroll
          for (int s = 0; s < KMAX; ++s) a[s] *= lds_load<double>(step_addr<PACK>(ado, s));
          wave_sync();
        }
        if constexpr (GRP) {
          if (pad) {
#pragma unroll
            for (int s = 0; s < KMAX; ++s) a[s] = 0;
#pragma unroll
            for (int j = 0; j < RPL; ++j) BB(j) = r[j] = DINV(j) = dgv[j] = 0;
          }
        }
        double bn2 = gsum<LANES>(ldot<RPL>(r, r));
        if constexpr (GRP) {
          bnc = __builtin_sqrt(bn2);
          bn2 = cross_cells<LANES>(bn2);
        }
        bn = __builtin_sqrt(bn2);
        tol2 = (P.rtol * bn) * (P.rtol * bn);
        double rr2 = bn2;  // ||r0||^2
        warm = use_x0 && finite(bn) && bn != 0.0;
        if (warm) {
#pragma unroll
          for (int j = 0; j < RPL; ++j) BB(j) = r[j] = t[j];
          rr2 = gsum<LANES>(ldot<RPL>(r, r));
        }
        it = 0;
        restarts_left = P.brs;
        restart();
        rho = rr2;  // (rhat, r) with rhat = r = r0
        active = true;
        if (!finite(bn)) {
          finish(kNonfinite, qnan());
        } else if (bn == 0.0) {
          finish(kConverged, 0.0);
        } else if (rr2 <= tol2) {
          finish(kConverged, __builtin_sqrt(rr2) / bn);  // the initial guess already meets rtol
        }
      }
    }
    if (__ballot(!dead) == 0ull) break;
    if (!active) continue;

    // ---- one BiCGStab iteration of this slot's cell ----
    // rho = (rhat, r) was reduced together with ||r||^2 at the end of the
    // previous iteration (or at staging / restart, where rhat = r).
    // Convergence tests compare squared norms with (rtol ||b||)^2.
    ++it;
    int ended = -1;  // -1 = continue, else kConverged / kBreakdown / kNonfinite
    if (!finite(rho)) {
      ended = kNonfinite;
    } else if (rho == 0.0) {
      ended = kBreakdown;
    } else {
      // After a start or restart p = v = 0 and rho_prev = alpha = omega = 1,
      // so this gives p = r on the first iteration without a separate branch.
      const double beta = qdiv(rho * alpha, rho_prev * omega);
#pragma unroll
      for (int j = 0; j < RPL; ++j) p[j] = r[j] + beta * (p[j] - omega * v[j]);
      sch.spmv(a, ad, xb, yb, gl, rows, p, v, dgv, span);
      double rhv[RPL];
      load_vec(RH, rhv);
      const double sigma = gsum<RL>(ldot<RPL>(rhv, v));
      if (!finite(sigma)) {
        ended = kNonfinite;
      } else if (sigma == 0.0) {
        ended = kBreakdown;
      } else {
        alpha = qdiv(rho, sigma);
#pragma unroll
        for (int j = 0; j < RPL; ++j) r[j] = r[j] - alpha * v[j];  // r now holds s
        // t = A s is formed before the half-step test so that ||s||^2,
        // (t, s) and (t, t) are reduced together (one reduction latency
        // instead of two; t is discarded on a half-step exit)
        sch.spmv(a, ad, xb, yb, gl, rows, r, t, dgv, span);
        double red3[3] = {ldot<RPL>(r, r), ldot<RPL>(t, t), ldot<RPL>(t, r)};
        gsum_n<RL>(red3);
        const double sn2 = red3[0], tt = red3[1], ts = red3[2];
        if (!finite(sn2)) {
          ended = kNonfinite;
        } else if (sn2 <= tol2) {
#pragma unroll
          for (int j = 0; j < RPL; ++j) XV(j) = XV(j) + alpha * p[j];
          ended = kConverged;
        } else if (!finite(tt)) {
          ended = kNonfinite;
        } else if (tt == 0.0) {
          ended = kBreakdown;
        } else {
          omega = qdiv(ts, tt);
#pragma unroll
          for (int j = 0; j < RPL; ++j) {
            XV(j) = XV(j) + alpha * p[j] + omega * r[j];
            r[j] = r[j] - omega * t[j];
          }
          // ||r||^2 of r = s - omega t with omega = (t, s) / (t, t) is
          // ||s||^2 - omega (t, s): only (rhat, r) needs a reduction.  (A
          // negative value from cancellation passes the test below; the true
          // residual then decides.)
          const double rn2 = sn2 - omega * ts;
          double rhr[RPL];
          load_vec(RH, rhr);
          const double rho_next = gsum<RL>(ldot<RPL>(rhr, r));
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
      // The true residual of the current iterate decides (t is free here).
      {
        double xv[RPL];
        load_vec(XV, xv);
        sch.spmv(a, ad, xb, yb, gl, rows, xv, t, dgv, span);
      }
#pragma unroll
      for (int j = 0; j < RPL; ++j) t[j] = BB(j) - t[j];
      const double tt2c = gsum<LANES>(ldot<RPL>(t, t));
      const double tt2 = GRP ? cross_cells<LANES>(tt2c) : tt2c;
      const double res = __builtin_sqrt(tt2) / bn;
      // GRP: the run's outcome, then each cell's own residual and status
      auto done = [&](int st) {
        if constexpr (GRP) {
          const double own = bnc > 0 ? __builtin_sqrt(tt2c) / bnc : 0.0;
          finish((st == kBreakdown || st == kNonfinite) ? st : (own <= P.rtol ? kConverged : kMaxit), own);
        } else {
          finish(st, res);
        }
      };
      if (ended == kNonfinite || !finite(res)) {
        done(kNonfinite);
      } else if (res <= P.rtol) {
        done(kConverged);
      } else if (it < P.maxit && ((ended == kConverged && P.rr) || (ended == kBreakdown && restarts_left > 0))) {
        if (ended == kBreakdown) --restarts_left;
#pragma unroll
        for (int j = 0; j < RPL; ++j) r[j] = t[j];
        restart();
        rho = tt2;  // (rhat, r) with rhat = r = b - A x
      } else {
        done(ended == kBreakdown ? kBreakdown : kMaxit);
      }
    }
  }

}

template <class S, int ADJ = -1, bool GRP = false, class MT = dev::NoMechTerms>
__device__ __forceinline__ void fp64_body(const KParams& P) {
  constexpr bool MECH = MT::kOn;
  extern __shared__ double lds[];
  // The schedule's value positions and the rows' diagonal positions, shared
  // by every cell slot of the workgroup, copied once into LDS.
  int32_t* ent_lds = (int32_t*)(lds + P.tbase);
  int32_t* diag_lds = ent_lds + S::KMAX * S::LANES;
  for (int i = threadIdx.x; i < S::KMAX * S::LANES; i += kWgThreads) ent_lds[i] = P.sched.ent[i];
  for (int i = threadIdx.x; i < P.n; i += kWgThreads) diag_lds[i] = P.diag_pos[i] & kEntPosMask;
  if (ADJ == 1 || (ADJ < 0 && P.adjoint)) {
    // the adjoint epilogue's (row, column) of every position
    uint32_t* coo = (uint32_t*)(lds + P.coobase);
    for (int i = threadIdx.x; i < P.nnz; i += kWgThreads)
      coo[i] = (uint32_t)(uint16_t)P.coo_row[i] | (uint32_t)(uint16_t)P.coo_col[i] << 16;
  }
  if constexpr (MECH) {
    // the shared rate constants, a zero, a one, and the kernel's J term program
    for (int i = threadIdx.x; i < P.mk; i += kWgThreads) lds[P.mtbase + i] = P.kr[i];
    if (threadIdx.x == 0) {
      lds[P.mtbase + P.mr] = 0.0;
      lds[P.mtbase + P.mr + 1] = 1.0;
    }
    int32_t* mt = (int32_t*)(lds + P.mtbase + P.mr + 2);
    for (int i = threadIdx.x; i < P.mtab_words; i += kWgThreads) mt[i] = P.mtab[i];
  }
  __syncthreads();
  const int wv = threadIdx.x >> 6;
  fp64_run<S, ADJ, GRP, MT>(P, lds, wv, ent_lds, diag_lds);
}

// Several mechanisms in one persistent launch.  Every wave drains the
// mechanisms' work queues in the given order (the host orders them by cost
// per cell, largest first), refilling its cell slots from the current queue;
// a wave moves to the next mechanism once the current queue is empty and its
// slots have finished.
template <int I, class S, class... Rest>
__device__ __forceinline__ void multi_run(const MultiParams& M, double* lds, int wv) {
  const int32_t* ent = (const int32_t*)(lds + M.ent_off[I]);
  fp64_run<S, 0>(M.m[I], lds, wv, ent, ent + S::KMAX * S::LANES);
  if constexpr (sizeof...(Rest) > 0) multi_run<I + 1, Rest...>(M, lds, wv);
}

template <class... Ss>
__device__ __forceinline__ void multi_body(const MultiParams& M) {
  extern __shared__ double lds[];
  constexpr int NM = sizeof...(Ss);
  constexpr int lanes[NM] = {Ss::LANES...};
  constexpr int ksteps[NM] = {Ss::KMAX...};
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    int32_t* e = (int32_t*)(lds + M.ent_off[m]);
    for (int i = threadIdx.x; i < ksteps[m] * lanes[m]; i += kWgThreads) e[i] = M.m[m].sched.ent[i];
    int32_t* dg = e + ksteps[m] * lanes[m];
    for (int i = threadIdx.x; i < M.m[m].n; i += kWgThreads) dg[i] = M.m[m].diag_pos[i] & kEntPosMask;
  }
  __syncthreads();
  const int wv = threadIdx.x >> 6;
  multi_run<0, Ss...>(M, lds, wv);
}

// Precompiled generic variant (segment boundaries read at run time).
template <int LANES, int RPL, int KMAX>
__global__ void __launch_bounds__(kWgThreads) k_fp64(KParams P) {
  fp64_body<dev::DynSched<LANES, RPL, KMAX>>(P);
}

#ifndef __HIPCC_RTC__
template <int LANES, int RPL, int KMAX>
hipError_t launch_fp64(const KParams& P, int grid, hipStream_t stream) {
  const size_t lds = ((size_t)P.tbase + ((size_t)KMAX * LANES + P.n + 1) / 2) * sizeof(double);
  hipLaunchKernelGGL((k_fp64<LANES, RPL, KMAX>), dim3(grid), dim3(kWgThreads), lds, stream, P);
  return hipGetLastError();
}
#endif

}  // namespace bcs
