// Definitions shared by the host code and the gfx950 kernels.  Safe to
// compile both with hipcc and with the runtime compiler (hipRTC), which has
// no standard headers.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#else
using __hip_internal::int16_t;
using __hip_internal::uint16_t;
using __hip_internal::int32_t;
using __hip_internal::int64_t;
using __hip_internal::uint32_t;
using __hip_internal::uint64_t;
using __hip_internal::uint8_t;
#endif

namespace bcs {

// per-cell status (values of BCS_CONVERGED .. BCS_NONFINITE)
constexpr int kConverged = 0;
constexpr int kMaxit = 1;
constexpr int kBreakdown = 2;
constexpr int kNonfinite = 3;
// matrix kinds (values of BCS_J_GAMMA, BCS_A_DIRECT)
constexpr int kJGamma = 0;
constexpr int kADirect = 1;

// Waves per workgroup of the solve kernels (a forward kernel compiled per
// pattern may be built with another count, BCS_WG_WAVES defined in its
// source).  Each wave works on its own cells with its own LDS slice; the
// waves synchronise once, at kernel start.
#ifndef BCS_WG_WAVES
#define BCS_WG_WAVES 4
#endif
constexpr int kWavesPerWg = BCS_WG_WAVES;
constexpr int kWgThreads = 64 * kWavesPerWg;

// Schedule entry: value position in the cell's CSR array, plus flags.
constexpr int32_t kEntDiag = 1 << 30;  // the entry is a diagonal position
constexpr int32_t kEntPad = 1 << 29;   // padding step (value 0; reads position 0)
constexpr int32_t kEntPosMask = kEntPad - 1;

// Schedule of one matrix (A, or A^T for the adjoint) for one lanes-per-cell
// choice.  Rows are dealt to (slot j, lane l) in the order of decreasing row
// length (a sliced-ELL layout with slice height = lanes per cell), so every
// slot j spans the same steps [seg_begin_j, seg_end_j) on every lane.
// Workspace of one solve (caller-owned device memory, 256-byte aligned):
// the work queue (word 0 hands out cell indices; kWsQueueBytes reserved),
// then the cost-order sort state (kOrderStateWords words), then the order
// itself (4 bytes per cell).  A clear kernel on the solve's stream zeroes the
// queue and the sort state before every solve.
constexpr int kQueueWords = 32;

// Per-lane vectors of a cell slot kept in its LDS state block by kernels
// built with kSchedLean (lane-major: vector k, row slot j, lane l at
// (k * RPL + j) * LANES + l), ahead of the SpMV result block: the iterate,
// the shadow residual, b and diag(A)^-1.
constexpr int kSlotX = 0;
constexpr int kSlotRhat = 1;
constexpr int kSlotB = 2;
constexpr int kSlotDinv = 3;
constexpr int kSlotVecs = 4;
constexpr int kWsQueueBytes = kQueueWords * 8;

// Cost order of the cells: a counting sort of the cells by a bucket of
// gamma (kOrderBuckets buckets of a quarter octave each, from 2^-16 up;
// larger gamma = stiffer cell = more iterations).  Queue position k then
// takes the cell of rank k/2 from the top for even k and from the bottom for
// odd k, so expensive cells start early while cheap ones keep the refill rate
// even.  The sort state is the bucket counts, then the bucket cursors.
constexpr int kOrderBuckets = 128;
// Cells a slot takes per claim when the cells come in a cost order.
constexpr int kClaimGroup = 2;
constexpr int kOrderStateWords = 2 * kOrderBuckets;
constexpr int kWsStateOffset = kWsQueueBytes;
constexpr int kWsOrderOffset = kWsStateOffset + kOrderStateWords * 4;

// Shapes of the specialised kernels' schedules (bits of their FLAGS).
// kSchedSpan: a lane whose slot-1 row is kRowSpan holds one long row over
// the steps of slots 0 and 1 together; slot 0 then yields a partial sum and
// slot 1 the rest, which the SpMV adds into slot 0.  kSchedDiag: the diagonal
// entries are not in the schedule; the SpMV starts each row's sum with the
// diagonal term, taken from the row's own operand value in registers.
constexpr int kSchedSpan = 1;
constexpr int kSchedDiag = 2;
// Register-saving options (not shapes), for kernels that hold several
// schedules: kSchedPack keeps two 16-bit gather addresses per VGPR even for
// short schedules (one VALU operation per step, half the registers);
// kSchedWin8 keeps 8 gathers in flight instead of kGatherChunk.
constexpr int kSchedPack = 4;
constexpr int kSchedWin8 = 8;
// kSchedLean: the FP64 body keeps the vectors of kSlotVecs in the slot's LDS
// state block instead of registers (the layout then gives every slot
// kSlotVecs + 1 blocks of RPL x LANES doubles).
constexpr int kSchedLean = 16;
constexpr int16_t kRowSpan = -2;
// A J term word 1: the other reactant (16 bits; kNoSpecies = none) | (S + 128) << 16 | factor 2 << 24.
constexpr int kNoSpecies = 0xffff;


struct DevSchedule {
  const int32_t* ent;   // [ksteps * lanes] value position | kEntDiag, or kEntPad
  const uint8_t* col;   // [ksteps * lanes] gathered vector index (row of the other operand)
  const int16_t* row;   // [rpl * lanes] row owned by slot j of lane l, -1 = none, kRowSpan = slot 0's row
  int32_t ksteps;       // steps per lane (sum of slot segment lengths)
  int32_t rpl;          // row slots per lane
  uint64_t flush[2];    // bit s set: a slot's segment ends after step s
};

// Everything a solve kernel needs, passed by value.
struct KParams {
  int64_t ncells;
  int32_t n, nnz;
  const double* values;
  const double* gamma;
  int64_t gamma_stride;
  const double* b;
  const double* x0;    // forward: initial guess [ncells, n], or null for x0 = 0
  const double* xin;   // adjoint: forward solution x
  double rtol;
  int32_t maxit;
  int32_t precond;
  int32_t kind;
  int32_t rr;
  int32_t brs;
  double inner_rtol;
  int32_t max_refine;
  int32_t budget;      // mixed form: 0 = maxit per inner solve, 1 = per cell over its inner solves
  int32_t grad_kind;   // adjoint: 0 = dL/dA, 1 = dL/d(values) (dL/dJ in J mode)
  double* x;           // solution (adjoint: lambda)
  double* grad_vals;   // adjoint only: gradient on the pattern (per grad_kind)
  double* grad_gamma;  // adjoint only, J mode: dL/dgamma per cell, or null
  int32_t* iters;
  double* resid;
  int32_t* status;
  int32_t* refinements;
  const int32_t* diag_pos;  // [n] CSR position of the diagonal (0 if absent)
  DevSchedule sched;        // schedule of the solved matrix (A, or A^T for the adjoint)
  const int16_t* coo_row;   // [nnz] row of each CSR position (adjoint gradient)
  const int16_t* coo_col;   // [nnz] column of each CSR position
  int32_t adjoint;          // 1: solve with A^T, write grad_b = lambda and grad_A
  unsigned long long* queue;  // claim counter (workspace word 0), zeroed before the launch; null: slot k solves cell k
  const int32_t* order;       // cells in decreasing cost order, or null for index order
  int64_t qfirst;             // > 0: slots' first claims take queue positions [0, qfirst) without the counter, which starts at qfirst
  // Workgroup LDS, in doubles: the operand block of slot g of wave w at
  // w * wxs + g * xs (the only region gathers address, kept below 64 KiB
  // for 16-bit addresses), its state block at bbase + w * wbs + g * bs, then
  // the schedule tables at tbase.  Per-wave strides keep the waves of a
  // multi-mechanism launch, which may be on different mechanisms at a time,
  // in disjoint regions.
  int32_t xs, wxs;          // operand block stride (n + spare, and a second n-vector for the adjoint), per wave
  int32_t bbase, bs, wbs;   // state blocks: start, stride, stride per wave
  int32_t yoff;             // offset of the SpMV result block (RPL x LANES) within the state block
  int32_t tbase;            // start of the schedule tables
  int32_t coobase;          // adjoint: start of the (row | column << 16) word of every position
  // ILU(0) preconditioning (kernels compiled per pattern only).  The strict
  // lower and strict upper parts of the factors each have their own
  // schedule (rows dealt by their own lengths); the factorization program
  // and the 16-bit value-position tables are copied into LDS at tbase.
  DevSchedule schedL, schedU;
  const uint16_t* ilu_tab;  // [KA*L | KL*L | KU*L | n + 1]: positions in the slot's factor block
  const uint32_t* fprog;    // factorization program (see ilu_factor), fprog_words words
  int32_t fprog_words;
  int32_t sweeps;           // Jacobi sweeps per triangular solve
  int32_t fs;               // slot block stride (doubles): the factor block, later the operand
  // Solves from a mechanism (kernels compiled with a dev::MechTerms): J is
  // assembled per cell from the concentrations y [ncells, n] and rate
  // constants (k[c * k_stride + r]) while the cell is staged, by the kernel's
  // J term program.  LDS from mtbase (doubles): the mr rate constants (copied
  // when shared: mk = mr, else mk = 0), a zero, a one, then the program, two
  // words per (term, lane): the LDS byte address of the term's rate constant
  // (of the zero for a padding term, of the one for a padding step's term; a
  // multiple of 8) | factor 2 (bit 0) | the byte offset of its y factor in the
  // operand block << 16; then the high word of S as a double (S is a small
  // integer: the low word is 0).
  const double* y;
  const double* kr;
  int64_t k_stride;
  const int32_t* mtab;
  int32_t mtab_words;
  int32_t mtbase, mk, mr;
  // Debug (bcs_debug_count_visits; kernels compiled with BCS_COUNT_VISITS
  // defined): every time a cell's outputs are written,
  // visits[cell] is incremented, so a test can check that the work queue
  // hands every cell out exactly once.  Null in normal use.
  int32_t* visits;
};

// ILU(0) factor block of a slot: the nnz values in CSR order, then three
// constant elements that the schedules and the factorization program use for
// padding (positions as in the 16-bit tables).
constexpr int kIluZero = 0;   // offset past nnz: always 0.0
constexpr int kIluUnit = 1;   // always 1.0 (divisor of ops on the upper part)
constexpr int kIluJunk = 2;   // target of padding ops
constexpr int kIluSpare = 3;  // elements after the nnz values

// Arguments of a multi-mechanism launch.
constexpr int kMaxMech = 8;
struct MultiParams {
  int32_t nmech;
  int32_t ent_off[kMaxMech];    // LDS offset (doubles) of each mechanism's schedule copy
  KParams m[kMaxMech];          // per-mechanism solve arguments (queue[0] = its work queue)
};

}  // namespace bcs
