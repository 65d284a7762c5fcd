// Device building blocks of the batched Block-cells solvers (gfx950, wave64).
//
// Layout of a cell on chip.  A cell is owned by LANES consecutive lanes of a
// wavefront (16, 32 or 64; 64/LANES cells per wave).  Rows are dealt to
// (slot j, lane l) by decreasing length, RPL slots per lane, so that slot j
// covers the same schedule steps on every lane: the matrix is held as a
// sliced-ELL block whose slice height is LANES.  The cell's matrix values
// live in VGPRs (a[s], one per schedule step), its Krylov vectors in VGPRs
// (one value per owned row), and only the SpMV operand is staged in the
// cell's LDS slice, from which every lane gathers its columns.
#pragma once

#include "bcs_kdefs.h"

namespace bcs {
namespace dev {

// Make this wave's LDS writes visible to its own later reads (and keep the
// compiler from moving LDS accesses across the point).  A wavefront's LDS
// instructions complete in order, so no s_barrier is needed.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Fused multiply-add in the operands' own precision (__builtin_fma is the
// double version: with float operands it would compute in FP64 and round
// twice).
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Lane exchange within 16-lane rows.  Every control used here reads a valid
// lane for every lane, so bound_ctrl never zeroes a lane; it only lets the
// move write its destination without first copying the source into it.
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}

// All-reduce sum over the LANES lanes of a cell.  Butterfly: every lane adds
// the same two partial sums (in either order, and IEEE addition commutes), so
// all lanes of the cell end with bitwise the same value, and the result of a
// cell never depends on which slot or wave it ran in.
// Sum of a value over 16-lane row pairs (0,1), (2,3) with v_permlane16_swap
// (SWAP32 = false), or over the two wave halves with v_permlane32_swap: both
// results of the swap applied to (v, v) hold the pair in the same order, so
// every lane adds the same two operands in the same order.
template <bool SWAP32>
__device__ __forceinline__ double pair_sum(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
  uint32_t a_lo, b_lo, a_hi, b_hi;
  if constexpr (SWAP32) {
    const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    a_lo = l[0], b_lo = l[1], a_hi = h[0], b_hi = h[1];
  } else {
    const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    a_lo = l[0], b_lo = l[1], a_hi = h[0], b_hi = h[1];
  }
  return __builtin_bit_cast(double, ((uint64_t)a_hi << 32) | a_lo) +
         __builtin_bit_cast(double, ((uint64_t)b_hi << 32) | b_lo);
}

template <bool SWAP32>
__device__ __forceinline__ float pair_sum(float v) {
  const uint32_t u = __builtin_bit_cast(uint32_t, v);
  uint32_t a, b;
  if constexpr (SWAP32) {
    const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    a = r[0], b = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    a = r[0], b = r[1];
  }
  return __builtin_bit_cast(float, a) + __builtin_bit_cast(float, b);
}

template <int LANES, typename T>
__device__ __forceinline__ T gsum(T v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);  // row_half_mirror: quads 0<->1 within each 8 lanes
  v += dpp<0x140>(v);  // row_mirror: halves 0<->1 within each 16-lane row
  if constexpr (LANES >= 32) v = pair_sum<false>(v);
  if constexpr (LANES >= 64) v = pair_sum<true>(v);
  return v;
}

// The levels of gsum<64> above LANES: from a value summed over each cell's
// LANES lanes to its sum over the whole wave (bitwise what gsum<64> gives).
template <int LANES, typename T>
__device__ __forceinline__ T cross_cells(T v) {
  if constexpr (LANES <= 16) v = pair_sum<false>(v);
  if constexpr (LANES <= 32) v = pair_sum<true>(v);
  return v;
}

// All-reduce K values at once, level by level: every value goes through
// exactly the steps of gsum (so each result is bitwise what gsum gives), and
// the independent butterflies interleave, each one's moves and adds filling
// the others' wait states.
template <int LANES, int K, typename T>
__device__ __forceinline__ void gsum_n(T (&v)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp<0xB1>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp<0x4E>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp<0x141>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp<0x140>(v[k]);
  if constexpr (LANES >= 32) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = pair_sum<false>(v[k]);
  }
  if constexpr (LANES >= 64) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = pair_sum<true>(v[k]);
  }
}

// Hide a wave-uniform value from the optimiser so that conditions derived
// from it are evaluated where they are used instead of being hoisted and kept
// live across the whole kernel (which exhausts the scalar registers).
template <typename T>
__device__ __forceinline__ T opaque(T v) {
  asm volatile("" : "+s"(v));
  return v;
}

// Copy a lane's packed words so that values unpacked from the copy are
// recomputed at this use instead of being hoisted and kept live unpacked.
template <int N>
__device__ __forceinline__ void opaque_inplace(uint32_t (&w)[N]) {
#pragma unroll
  for (int q = 0; q < N; ++q) asm volatile("" : "+v"(w[q]));
}

template <int N>
__device__ __forceinline__ void opaque_copy(const uint32_t (&in)[N], uint32_t (&out)[N]) {
#pragma unroll
  for (int q = 0; q < N; ++q) {
    out[q] = in[q];
    asm volatile("" : "+v"(out[q]));
  }
}

// Loads through 32-bit LDS byte addresses.  The gather addresses are kept as
// absolute LDS addresses so that a gather is one ds_read with no address
// arithmetic.
typedef __attribute__((address_space(3))) char lds_char_t;

__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)(__UINTPTR_TYPE__)(const lds_char_t*)p;
}

template <typename T>
__device__ __forceinline__ T lds_load(uint32_t addr) {
  return *(const __attribute__((address_space(3))) T*)(__UINTPTR_TYPE__)addr;
}

// LDS byte address of step s: PACK = 2 packs two 16-bit addresses per word
// (saves VGPRs, costs one VALU op per step), PACK = 1 keeps one per word.
template <int PACK, int N>
__device__ __forceinline__ uint32_t step_addr(const uint32_t (&ad)[N], int s) {
  if constexpr (PACK == 1) return ad[s];
  return (s & 1) ? (ad[s >> 1] >> 16) : (ad[s >> 1] & 0xffffu);
}

// Fill a lane's address words for schedule `col` (steps x lanes, step-major)
// and a cell slot whose operand starts at LDS byte address `base`.
template <int PACK, int KMAX, int LANES, int N>
__device__ __forceinline__ void build_addr(uint32_t (&ad)[N], const uint8_t* col, uint32_t base, int gl) {
#pragma unroll
  for (int q = 0; q < N; ++q) {
    uint32_t w = 0;
#pragma unroll
    for (int i = 0; i < PACK; ++i) {
      const int s = PACK * q + i;
      if (s < KMAX) w |= (base + (uint32_t)col[s * LANES + gl] * 8u) << (16 * i);
    }
    ad[q] = w;
  }
}

__device__ __forceinline__ bool flush_bit(uint64_t f0, uint64_t f1, int s) {
  return s < 64 ? ((f0 >> s) & 1ull) != 0 : ((f1 >> (s - 64)) & 1ull) != 0;
}

constexpr int kGatherChunk = 16;

// J terms evaluated together when a kernel assembles J while staging a cell.
constexpr int kJTermChunk = 8;

// Slots are numbered workgroup by workgroup, wave by wave, slot by slot.
__device__ __forceinline__ int64_t slot_index(int wv, int grp, int slots_per_wave) {
  return ((int64_t)blockIdx.x * kWavesPerWg + wv) * slots_per_wave + grp;
}

// held[0] of a slot whose first claim is handed out without the counter.
constexpr int32_t kFirstClaim = -2;

// A slot's held[0] at kernel start.  Without a work queue (queue null: the
// launch has a slot for every cell) slot k takes cell k, -1 if there is no
// such cell.  With a queue whose counter starts at qfirst > 0, the slots'
// first claims take the positions below qfirst without the counter
// (kFirstClaim; slot k from k * cells per claim).  Else -1.
__device__ __forceinline__ int32_t initial_held(const unsigned long long* queue, int64_t qfirst, int64_t ncells, int wv,
                                                int grp, int slots_per_wave) {
  if (queue) return qfirst > 0 ? kFirstClaim : -1;
  const int64_t c = slot_index(wv, grp, slots_per_wave);
  return c < ncells ? (int32_t)c : -1;
}

// Claim the next cell for a slot (LANES lanes starting at lane `leader`):
// one atomic on the queue's claim counter by the slot's first lane,
// broadcast to the slot.  Returns false once every cell has been handed out.
// In index order a claim takes one queue position, the cell of that index.
// With a cost order a claim takes kClaimGroup consecutive positions, whose
// cells (queue position k is the cell of rank k/2 from the expensive end for
// even k, from the cheap end for odd k) are read from the order in one
// memory round trip; the first is solved now, the others are kept in
// held[] (-1 when none) and solved next without another claim.  Without a
// queue (null: the launch has a slot for every cell) a slot solves only the
// cell initial_held put in held[0].  A slot whose held[0] is kFirstClaim
// takes its first claim's positions from its slot index (wv, grp,
// slots_per_wave) instead of the counter (FIRST: kernels built without that
// path, whose launches always start the counter at 0, leave it out).
template <bool FIRST = true>
__device__ __forceinline__ bool claim_cell(unsigned long long* queue, const int32_t* order, int64_t ncells,
                                           int leader, bool is_leader, int64_t& cell,
                                           int32_t (&held)[kClaimGroup - 1], int wv, int grp, int slots_per_wave) {
  if (held[0] >= 0) {
    cell = held[0];
#pragma unroll
    for (int q = 0; q + 1 < kClaimGroup - 1; ++q) held[q] = held[q + 1];
    held[kClaimGroup - 2] = -1;
    return true;
  }
  if (!queue) return false;
  unsigned long long c = 0;
  if (FIRST && held[0] == kFirstClaim) {
    c = (unsigned long long)slot_index(wv, grp, slots_per_wave) * (order ? kClaimGroup : 1);
    held[0] = -1;
  } else {
    if (is_leader) c = atomicAdd(queue, order ? (unsigned long long)kClaimGroup : 1ull);
    c = __shfl(c, leader, 64);
  }
  if (c >= (unsigned long long)ncells) return false;
  if (order) {
    int32_t v[kClaimGroup];
#pragma unroll
    for (int q = 0; q < kClaimGroup; ++q) {
      const int64_t k = (int64_t)c + q;
      const int64_t rank = (k & 1) ? ncells - 1 - (k >> 1) : (k >> 1);
      v[q] = -1;
      if (is_leader && k < ncells) v[q] = order[rank];
    }
    cell = (int64_t)__shfl(v[0], leader, 64);
#pragma unroll
    for (int q = 1; q < kClaimGroup; ++q) held[q - 1] = __shfl(v[q], leader, 64);
  } else {
    cell = (int64_t)c;
  }
  return true;
}

// Schedule policies.  Both run out = M * in for the cell's matrix held as
// schedule values a[] (this lane's KMAX steps) and packed LDS byte addresses
// ad[] (absolute LDS byte addresses, one or two 16-bit addresses per word).
// `in` and `out` are this lane's owned rows (padding rows are staged into the
// spare element n of the slice); xb is the cell's operand slice and yb its
// result slice (RPL x LANES, slot-major).  Gathers are issued a chunk at a time, ahead
// of the chunk's FMAs.

// Slot boundaries known only at run time (precompiled generic variants): the
// steps of slot j end where bit s of (f0, f1) is set; the finished row sum is
// written to yb[j*LANES + lane] (a uniform branch around one LDS store, so no
// register array is indexed at run time) and read back at the end.
template <int LANES_, int RPL_, int KMAX_>
struct DynSched {
  static constexpr int LANES = LANES_, RPL = RPL_, KMAX = KMAX_;
  static constexpr int PACK = 2, NW = (KMAX + 1) / 2;
  static constexpr int FLAGS = 0;  // plain sliced-ELL schedules only
  uint64_t f0_, f1_;
  __device__ explicit DynSched(const DevSchedule& d) : f0_(d.flush[0]), f1_(d.flush[1]) {}

  // T = double, or float stored in the low half of double-spaced slots
  // (so both precisions share the slot layout and the gather addresses).
  template <typename T>
  __device__ __forceinline__ void spmv(const T (&a)[KMAX], const uint32_t (&ad_)[NW], double* xb,
                                       double* yb, int gl, const int (&rows)[RPL], const T (&in)[RPL],
                                       T (&out)[RPL], const T (&)[RPL] = {}, T = T(0)) const {
    const uint64_t f0 = opaque(f0_), f1 = opaque(f1_);
    uint32_t ad[NW];
    opaque_copy<NW>(ad_, ad);
#pragma unroll
    for (int j = 0; j < RPL; ++j) *(T*)(xb + rows[j]) = in[j];
    wave_sync();
    T acc = 0;
    double* ydst = yb + gl;
#pragma unroll
    for (int s0 = 0; s0 < KMAX; s0 += kGatherChunk) {
      constexpr int C = kGatherChunk;
      T g[C];
#pragma unroll
      for (int i = 0; i < C; ++i) {
        const int s = s0 + i;
        if (s < KMAX) g[i] = lds_load<T>(step_addr<PACK>(ad, s));
      }
#pragma unroll
      for (int i = 0; i < C; ++i) {
        const int s = s0 + i;
        if (s < KMAX) {
          acc = fmat(a[s], g[i], acc);
          if (flush_bit(f0, f1, s)) {
            *(T*)ydst = acc;
            ydst += LANES;
            acc = 0;
          }
        }
      }
    }
    wave_sync();
#pragma unroll
    for (int j = 0; j < RPL; ++j) out[j] = *(const T*)(yb + j * LANES + gl);
    wave_sync();
  }
};

// Slot segment lengths known at compile time (kernels compiled for one
// pattern at plan creation): straight-line code, row sums land directly in
// out[j].
template <int LANES_, int FLAGS_, int... SEG>
struct StaticSched {
  static constexpr int LANES = LANES_;
  static constexpr int FLAGS = FLAGS_;
  static constexpr bool SPAN = (FLAGS & kSchedSpan) != 0, DIAG = (FLAGS & kSchedDiag) != 0;
  static constexpr int RPL = sizeof...(SEG);
  static_assert(!SPAN || RPL >= 2, "a spanning row needs two slots");
  static constexpr int KMAX = (SEG + ...);
  // short schedules keep one address per word (no extraction on the hot path)
  static constexpr int PACK = (KMAX <= 48 && (FLAGS & kSchedPack) == 0) ? 1 : 2, NW = (KMAX + PACK - 1) / PACK;
  __device__ explicit StaticSched(const DevSchedule&) {}

  // slot of step s, and whether s is the last step of its slot
  static constexpr int slot_of(int s) {
    constexpr int seg[RPL] = {SEG...};
    int e = 0;
    for (int j = 0; j < RPL; ++j) {
      e += seg[j];
      if (s < e) return j;
    }
    return RPL - 1;
  }
  static constexpr int slot_start(int s) {
    constexpr int seg[RPL] = {SEG...};
    int b = 0;
    for (int j = 0; j < RPL; ++j) {
      if (s < b + seg[j]) return b;
      b += seg[j];
    }
    return b;
  }
  static constexpr bool ends_slot(int s) {
    constexpr int seg[RPL] = {SEG...};
    int e = 0;
    for (int j = 0; j < RPL; ++j) {
      e += seg[j];
      if (s == e - 1) return true;
    }
    return false;
  }

  // out = A in over the schedule.  dg (DIAG): each owned row's diagonal
  // value, whose term starts the row's sum.  sm (SPAN): 1 on a lane whose
  // slots 0 and 1 hold one row (slot 1's sum is added into slot 0 and slot
  // 1, a padding row, ends 0), else 0.
  // STAGE = false: `in` is already in the operand block (every owned row,
  // and 0 in the spare element), so the stores are skipped.
  template <typename T, bool STAGE = true>
  __device__ __forceinline__ void spmv(const T (&a)[KMAX], uint32_t (&ad)[NW], double* xb,
                                       double* /*yb*/, int /*gl*/, const int (&rows)[RPL], const T (&in)[RPL],
                                       T (&out)[RPL], const T (&dg)[RPL], T sm) const {
    opaque_inplace<NW>(ad);
    if constexpr (STAGE) {
#pragma unroll
      for (int j = 0; j < RPL; ++j) *(T*)(xb + rows[j]) = in[j];
      wave_sync();
    }
    // two accumulators per slot (even / odd steps of the slot) halve the
    // FMA dependency chain; gathers run kGatherChunk (kSchedWin8: 8) steps
    // ahead of the FMAs that consume them
    constexpr int W = (FLAGS & kSchedWin8) ? 8 : kGatherChunk;
    T acc0 = DIAG ? dg[0] * in[0] : T(0), acc1 = 0;
    T g[W];
    // The SIMD's other wave is usually in its reductions or updates: while
    // this wave gathers, it issues first (measured 0.8% faster on the n = 80
    // workload; raising the reductions' priority as well lost that again).
    __builtin_amdgcn_s_setprio(2);
#pragma unroll
    for (int s = 0; s < W; ++s)
      if (s < KMAX) g[s] = lds_load<T>(step_addr<PACK>(ad, s));
#pragma unroll
    for (int s = 0; s < KMAX; ++s) {
      const T gv = g[s % W];
      if (s + W < KMAX) g[s % W] = lds_load<T>(step_addr<PACK>(ad, s + W));
      if (((s - slot_start(s)) & 1) == 0)
        acc0 = fmat(a[s], gv, acc0);
      else
        acc1 = fmat(a[s], gv, acc1);
      if (ends_slot(s)) {
        constexpr int last = RPL - 1;
        const int j = slot_of(s);
        const int jn = j < last ? j + 1 : last;
        out[j] = acc0 + acc1;
        acc0 = (DIAG && j < last) ? dg[jn] * in[jn] : T(0);
        acc1 = 0;
      }
    }
    __builtin_amdgcn_s_setprio(0);
    if constexpr (SPAN) {
      out[0] = fmat(sm, out[1], out[0]);
      out[1] = (T(1) - sm) * out[1];
    }
    wave_sync();
  }

  // Plain schedules (the mixed form's kernels): no diagonal or span terms.
  template <typename T>
  __device__ __forceinline__ void spmv(const T (&a)[KMAX], uint32_t (&ad)[NW], double* xb, double* yb, int gl,
                                       const int (&rows)[RPL], const T (&in)[RPL], T (&out)[RPL]) const {
    static_assert(FLAGS == 0, "this schedule needs the diagonal and span terms");
    const T none[RPL] = {};
    spmv(a, ad, xb, yb, gl, rows, in, out, none, T(0));
  }
};

template <int RPL, typename T>
__device__ __forceinline__ T ldot(const T (&u)[RPL], const T (&v)[RPL]) {
  T s = 0;
#pragma unroll
  for (int j = 0; j < RPL; ++j) s = fmat(u[j], v[j], s);
  return s;
}

// a / b for finite, nonzero b of normal magnitude (the iteration's scalars,
// checked before they divide): the hardware reciprocal estimate refined by one
// Newton step, then one correction of the quotient from its residual
// a - b q.  Within about an ulp of the rounded quotient, in six dependent
// operations instead of the scaled IEEE division sequence.
__device__ __forceinline__ double qdiv(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = __builtin_fma(__builtin_fma(-b, r, 1.0), r, r);
  const double q = a * r;
  return __builtin_fma(__builtin_fma(-b, q, a), r, q);
}

// The same in FP32 (the mixed form's inner solve): the FP32 reciprocal is
// accurate to about an ulp, so one quotient correction suffices.
__device__ __forceinline__ float qdiv(float a, float b) {
  const float r = __builtin_amdgcn_rcpf(b);
  const float q = a * r;
  return __builtin_fmaf(__builtin_fmaf(-b, q, a), r, q);
}

// A quiet NaN materialised where it is used (from a scalar register), so
// that the constant is not kept live in vector registers across the solve
// loop for the rare non-finite exit.
__device__ __forceinline__ double qnan() {
  return __builtin_bit_cast(double, opaque<uint64_t>(0x7ff8000000000000ull));
}

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }
__device__ __forceinline__ bool finite(float v) { return __builtin_isfinite(v); }

// Shape of the J term program of a kernel that assembles J while staging a
// cell: first the J0 terms of CSR position 0, which every lane evaluates (a
// padding step of the schedule takes that value, as the plain kernel loads
// position 0 for it), then the lane's KMAX schedule positions and its RPL
// rows' diagonal positions, and for each of these P positions the number of
// terms T[p] every lane evaluates (the largest count among the lanes;
// shorter lists are padded with terms that add nothing).  The program
// itself, two words per (term, lane), is data (KParams::mtab); its shape is
// compiled in so that every term's LDS address is a constant offset.
template <int J0, int... T>
struct MechTerms {
  static constexpr bool kOn = true;
  static constexpr int kJ0 = J0;
  static constexpr int kP = sizeof...(T);
  static constexpr int count(int p) {
    constexpr int t[] = {T...};
    return t[p];
  }
  static constexpr int start(int p) {
    constexpr int t[] = {T...};
    int s = 0;
    for (int i = 0; i < p; ++i) s += t[i];
    return s;
  }
  static constexpr int total() { return (0 + ... + T); }
  // position of term u of the lane's program (terms numbered across positions)
  static constexpr int pos_of(int u) {
    constexpr int t[] = {T...};
    int p = 0;
    while (u >= t[p]) u -= t[p++];
    return p;
  }
};
struct NoMechTerms {
  static constexpr bool kOn = false;
  static constexpr int kJ0 = 0;
  static constexpr int kP = 0;
};

// Calls f(Pos<I>{}) for I = I0 .. N-1, each with its index as a constant.
template <int V>
struct Pos {
  static constexpr int value = V;
};
template <int I, int N, class F>
__device__ __forceinline__ void for_pos(F&& f) {
  if constexpr (I < N) {
    f(Pos<I>{});
    for_pos<I + 1, N>(f);
  }
}

}  // namespace dev
}  // namespace bcs
