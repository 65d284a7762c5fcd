// Host side of the library: pattern validation, schedule construction, kernel
// selection (precompiled variants, or pattern-specialised kernels compiled at
// plan creation), the layout autotuner, plan objects and the C-ABI entry
// points declared in include/bcs.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "bcs_internal.h"

namespace {

thread_local std::string g_err;
thread_local int32_t* g_visits = nullptr;  // bcs_debug_count_visits

int fail(int code, const char* fmt, ...) {
  char buf[640];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(BCS_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

bool verbose() { return std::getenv("BCS_VERBOSE") != nullptr; }

// Host form of a schedule (see DevSchedule).
struct HostSchedule {
  int lanes = 0, rpl = 0, ksteps = 0;
  std::vector<int> seg;  // slot segment lengths
  int flags = 0;         // kSchedSpan / kSchedDiag (specialised kernels)
  std::vector<int32_t> ent;
  std::vector<uint8_t> col;
  std::vector<int16_t> row;
  uint64_t flush[2] = {0, 0};
};

// Deal the rows of a CSR matrix (rp, ci; entry k stores value position
// pos[k]) to `rpl` slots of `lanes` lanes, longest rows first, and list each
// lane's entries slot after slot.  Slot j spans the same LEN_j steps on every
// lane, LEN_j = longest row in the slot (at least 1); shorter rows and absent
// rows are padded with entries that gather the slot's spare operand element
// n, which is always 0.  If kmax > 0
// the last slot is extended so that every lane runs exactly kmax steps (the
// precompiled variants); kmax = 0 keeps the natural length (specialised
// kernels).  ksteps > kmax on return means the pattern does not fit.
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
  if (kmax > 0) {
    if (ks > kmax) return S;
    len[rpl - 1] += kmax - ks;
    ks = kmax;
    S.ksteps = ks;
  }
  S.seg = len;
  S.ent.assign((size_t)ks * lanes, bcs::kEntPad);
  S.col.assign((size_t)ks * lanes, (uint8_t)n);  // padding gathers the slot's spare element, always 0
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
    else if (last < 128)
      S.flush[1] |= 1ull << (last - 64);
    s0 += len[j];
  }
  return S;
}

// Schedule of a specialised kernel.  As build_schedule with kmax = 0, with
// two optional shapes (allowed: mask of kSchedDiag / kSchedSpan):
// - kSchedDiag (every row holds its diagonal): the diagonal entries are left
//   out; the kernel starts each row's sum with the diagonal term instead.
// - kSchedSpan: the nx longest rows each take slots 0 and 1 of one lane
//   (lanes 0 .. nx-1, slot-1 row kRowSpan), the other rows fill slots 0 and 1
//   of the remaining lanes and the later slots of every lane, longest first.
//   A few long rows then no longer set the length of slot 0 for every lane;
//   nx is chosen for the fewest steps (nx = 0, the plain deal, if none is
//   shorter).
// Returns ksteps = -1 if the result fails its own consistency check.
HostSchedule build_schedule_jit(int n, const std::vector<int>& rp, const std::vector<int>& ci,
                                const std::vector<int>& pos, int lanes, int rpl, int allowed) {
  bool diag_all = true;
  for (int i = 0; i < n && diag_all; ++i) {
    bool has = false;
    for (int k = rp[i]; k < rp[i + 1]; ++k) has |= ci[k] == i;
    diag_all = has;
  }
  const bool split = (allowed & bcs::kSchedDiag) && diag_all;
  auto kept = [&](int k, int i) { return !(split && ci[k] == i); };
  std::vector<int> len(n, 0);
  for (int i = 0; i < n; ++i)
    for (int k = rp[i]; k < rp[i + 1]; ++k) len[i] += kept(k, i);
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int u, int v) { return len[u] > len[v]; });

  // slot lengths with nx spanning lanes; 0 if the rows do not fit
  auto deal = [&](int nx, std::vector<int>& seg) -> int {
    seg.assign(rpl, 1);
    int q = nx;
    for (int j = 0; j < rpl; ++j) {
      const int cap = j < 2 ? lanes - nx : lanes;
      for (int c = 0; c < cap && q < n; ++c, ++q) seg[j] = std::max(seg[j], len[order[q]]);
    }
    if (q < n) return 0;
    if (nx > 0 && len[order[0]] > seg[0] + seg[1]) seg[1] = len[order[0]] - seg[0];
    int total = 0;
    for (int v : seg) total += v;
    return total;
  };
  std::vector<int> seg;
  int ks = deal(0, seg), nx = 0;
  if ((allowed & bcs::kSchedSpan) && rpl >= 2)
    for (int c = 1; c < lanes && c < n; ++c) {
      std::vector<int> sc;
      const int t = deal(c, sc);
      if (t > 0 && t < ks) {
        ks = t;
        seg = sc;
        nx = c;
      }
    }

  HostSchedule S;
  S.lanes = lanes;
  S.rpl = rpl;
  S.seg = seg;
  S.ksteps = ks;
  S.flags = (split ? bcs::kSchedDiag : 0) | (nx > 0 ? bcs::kSchedSpan : 0);
  S.row.assign((size_t)rpl * lanes, -1);
  int q = 0;
  for (int l = 0; l < nx; ++l, ++q) {
    S.row[l] = (int16_t)order[q];
    S.row[lanes + l] = bcs::kRowSpan;
  }
  for (int j = 0; j < rpl; ++j)
    for (int l = j < 2 ? nx : 0; l < lanes && q < n; ++l, ++q) S.row[(size_t)j * lanes + l] = (int16_t)order[q];
  S.ent.assign((size_t)ks * lanes, bcs::kEntPad);
  S.col.assign((size_t)ks * lanes, (uint8_t)n);  // padding gathers the slot's spare element, always 0
  int s0 = 0;
  for (int j = 0; j < rpl; ++j) {
    for (int l = 0; l < lanes; ++l) {
      const int i = S.row[(size_t)j * lanes + l];
      if (i < 0) continue;
      int t = 0;
      for (int k = rp[i]; k < rp[i + 1]; ++k) {
        if (!kept(k, i)) continue;
        const size_t at = (size_t)(s0 + t) * lanes + l;
        S.ent[at] = pos[k] | (ci[k] == i ? bcs::kEntDiag : 0);
        S.col[at] = (uint8_t)ci[k];
        ++t;
      }
    }
    const int last = s0 + seg[j] - 1;
    if (last < 64)
      S.flush[0] |= 1ull << last;
    else if (last < 128)
      S.flush[1] |= 1ull << (last - 64);
    s0 += seg[j];
  }

  // Check: every entry placed is a kept entry of the row that owns its lane
  // and step (a spanning row owns slots 0 and 1), with its own column, and
  // every kept entry is placed exactly once.
  const int nnz = rp[n];
  std::vector<int> inv(nnz, -1), seen(nnz, 0);
  for (int k = 0; k < nnz; ++k)
    if (pos[k] >= 0 && pos[k] < nnz) inv[pos[k]] = k;
  int placed = 0;
  for (int l = 0; l < lanes; ++l)
    for (int j = 0, b = 0; j < rpl; b += seg[j], ++j) {
      const int i = S.row[(size_t)j * lanes + l];
      for (int st = b; st < b + seg[j]; ++st) {
        const int32_t e = S.ent[(size_t)st * lanes + l];
        if (e & bcs::kEntPad) continue;
        const int owner = (i == bcs::kRowSpan) ? S.row[l] : i;
        const int k = inv[e & bcs::kEntPosMask];
        if (owner < 0 || k < rp[owner] || k >= rp[owner + 1] || !kept(k, owner) ||
            S.col[(size_t)st * lanes + l] != ci[k] || seen[k]++) {
          S.ksteps = -1;
          return S;
        }
        ++placed;
      }
    }
  int want = 0;
  for (int i = 0; i < n; ++i) want += len[i];
  if (placed != want) S.ksteps = -1;
  return S;
}

// Workgroup LDS layout, in doubles (the fields of KParams).  First one
// operand block per cell slot: the SpMV operand (n values plus a spare
// element that padding rows write to; the adjoint also stages lambda there
// for its gradient).  Gathers address only these blocks, through 16-bit byte
// addresses, so they must end below 64 KiB; their stride is 8 mod 32 doubles
// so that the slots of a wave start on different LDS banks.  Then one state
// block per slot: the SpMV result block (RPL x LANES) of the precompiled
// kernels.  Then the tables: the schedule's value
// positions (ksteps x lanes) and the diagonal's position in every row (n),
// 32-bit words.
struct WgLayout {
  int xs = 0, wxs = 0, bbase = 0, bs = 0, wbs = 0, yoff = 0, tbase = 0;
  int coobase = 0;  // adjoint kernels: each position's (row, column), after the tables
  size_t operand_bytes = 0, bytes = 0;
};

int slots_per_wg(int lanes) { return bcs::kWavesPerWg * (64 / lanes); }

// operand block stride and state block size of one slot (lean: the slot
// vectors of kSchedLean kernels ahead of the SpMV result block)
void slot_sizes(int n, int lanes, int rpl, bool lean, int* xs, int* bs) {
  const int xn = ((n + 1 + 7) / 8) * 8;
  *xs = ((xn + 31) / 32) * 32 + 8;
  *bs = (lean ? bcs::kSlotVecs + 1 : 1) * rpl * lanes;
}

size_t table_doubles(int n, int lanes, int ksteps) { return ((size_t)ksteps * lanes + (size_t)n + 1) / 2; }

WgLayout wg_layout(int n, int lanes, int rpl, int ksteps, int adjoint, bool lean = false,
                   int wpw = bcs::kWavesPerWg, int nnz = 0) {
  WgLayout L;
  slot_sizes(n, lanes, rpl, lean, &L.xs, &L.bs);
  L.yoff = lean ? bcs::kSlotVecs * rpl * lanes : 0;
  L.wxs = (64 / lanes) * L.xs;
  L.wbs = (64 / lanes) * L.bs;
  L.bbase = wpw * L.wxs;
  L.tbase = L.bbase + wpw * L.wbs;
  L.operand_bytes = (size_t)L.bbase * sizeof(double);
  L.bytes = ((size_t)L.tbase + table_doubles(n, lanes, ksteps)) * sizeof(double);
  if (adjoint) {
    // the gradient epilogue's table: row | column << 16 of every position
    L.coobase = (int)(L.tbase + table_doubles(n, lanes, ksteps));
    L.bytes += (((size_t)nnz + 1) / 2) * sizeof(double);
  }
  return L;
}

// LDS a workgroup may allocate: the device's limit, and at most 64 KiB
// (the layouts are tested up to that size).
size_t device_max_lds() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                                               hipSuccess || v <= 0)
    return 65536;
  return std::min<size_t>((size_t)v, 65536);
}

// The device's whole LDS per workgroup (160 KiB on gfx950), for kernels
// whose region beyond the first 64 KiB is read through 32-bit addresses
// only: the J term program of the kernels that assemble J.
size_t device_lds_limit() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                                               hipSuccess || v <= 0)
    return 65536;
  return (size_t)v;
}

bool layout_fits(const WgLayout& L) { return L.operand_bytes <= 65536 && L.bytes <= device_max_lds(); }

// Whether a specialised kernel of ksteps steps and rpl rows per lane is worth
// compiling: the lane's matrix values (2 VGPRs a step), gather addresses
// (half a VGPR a step) and register-resident vectors (8 VGPRs a row) must
// leave room in the 256 VGPRs of a wave; larger layouts would spill.
bool jit_feasible(int ksteps, int rpl) { return 2 * ksteps + (ksteps + 1) / 2 + 8 * rpl <= 240; }

// One launchable solve kernel with its schedule on the device.
struct Kernel {
  int lanes = 0, rpl = 0, ksteps = 0, adjoint = 0;
  std::vector<int> seg;               // slot segment lengths (specialised kernels)
  int flags = 0;                      // schedule shape (specialised kernels)
  int mtbase = 0;                     // kernels that assemble J: LDS offset (doubles) of the rate constants,
  std::vector<int> mterms;            // the J term program's shape (terms per position),
  int mwords = 0;                     // its size in 32-bit words
  void* mbuf = nullptr;               // and its device copy
  bool occ = false;                   // built with extra schedule flags for more waves per SIMD
  int occ_flags = 0;                  // those flags (kSchedLean | kSchedPack [| kSchedWin8])
  int waves = 0;                      // waves per SIMD the build asked for (0 = the compiler's choice)
  int wpw = bcs::kWavesPerWg;         // waves per workgroup
  const bcs::Variant* var = nullptr;  // precompiled variant, or
  bcs::JitKernel jit;                 // specialised kernel
  int max_blocks = 1;                 // resident workgroups per CU
  size_t lds = 0;
  WgLayout layout;
  bcs::DevSchedule d{};
  void* buf = nullptr;  // device schedule arrays
  // ILU(0) kernels (bcs_ilu.h): the triangles' schedules, the 16-bit value
  // position tables and the factorisation program (device copies in ibuf)
  bool ilu = false;
  int fs = 0, sweeps = 0, fprog_words = 0;
  bcs::DevSchedule dL{}, dU{};
  const uint16_t* ilu_tab = nullptr;
  const uint32_t* fprog = nullptr;
  void* ibuf = nullptr;

  hipError_t launch(const bcs::KParams& P, int grid, hipStream_t stream) const {
    if (var) return var->fp64(P, grid, stream);
    bcs::KParams copy = P;
    void* args[] = {&copy};
    return hipModuleLaunchKernel(jit.fn, grid, 1, 1, 64 * wpw, 1, 1, (unsigned)lds, stream, args, nullptr);
  }
};

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

int upload_schedule(const HostSchedule& S, Kernel* K) {
  const size_t ne = S.ent.size();
  const size_t bytes = ne * 4 + ne + S.row.size() * 2 + 64;
  void* buf = nullptr;
  HIP_TRY(hipMalloc(&buf, bytes));
  K->buf = buf;
  char* p = (char*)buf;
  HIP_TRY(hipMemcpy(p, S.ent.data(), ne * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p + ne * 4, S.row.data(), S.row.size() * 2, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p + ne * 4 + S.row.size() * 2, S.col.data(), ne, hipMemcpyHostToDevice));
  K->d.ent = (const int32_t*)p;
  K->d.row = (const int16_t*)(p + ne * 4);
  K->d.col = (const uint8_t*)(p + ne * 4 + S.row.size() * 2);
  K->d.ksteps = S.ksteps;
  K->d.rpl = S.rpl;
  K->d.flush[0] = S.flush[0];
  K->d.flush[1] = S.flush[1];
  return BCS_OK;
}

void free_kernel(Kernel* K) {
  if (K->buf) (void)hipFree(K->buf);
  if (K->ibuf) (void)hipFree(K->ibuf);
  if (K->mbuf) (void)hipFree(K->mbuf);
  K->buf = nullptr;
  K->ibuf = nullptr;
  K->mbuf = nullptr;
}

// J term program of a kernel that assembles J while staging a cell (the
// mechanism's J gather lists rearranged for the kernel's schedule).  Every
// lane first evaluates CSR position 0 (terms[0] terms): the plain kernel
// loads position 0's value for a padding step of the schedule, and the J
// kernel keeps that value in the slot's operand block for them.  Then lane l
// evaluates P = ksteps + rpl positions: the value position of each of its
// schedule steps (a padding step: one term that takes the kept value), then
// the diagonal position of each of its rows (nothing for a padding row,
// whose diagonal the staging code discards).  Position p has terms[1 + p]
// terms on every lane, the largest count among the lanes; entry (t, l) of
// the program is the word pair t * lanes + l (terms numbered from position 0
// on): the LDS byte address of the term's rate constant (the rate constants
// sit at mtbase doubles, followed by a zero that padding terms read and a
// one) | factor 2 in bit 0 | the byte offset of the y factor in the cell's
// operand block (the other reactant; element n + 1, which holds 1, for a
// first-order term and for padding; element n + 2 for the kept position-0
// value) << 16, then the high word of S as a double (0 for padding).  False
// if the constants lie beyond 16-bit LDS addresses.
bool mech_program(const HostSchedule& S, int n, int lanes, int rpl, const std::vector<int>& rp,
                  const std::vector<int>& ci, const bcs_mechanism& m, int mtbase, std::vector<int>* terms,
                  std::vector<int32_t>* prog) {
  if ((size_t)(mtbase + m.R + 2) * sizeof(double) > 65536) return false;
  std::vector<int> diag(n, 0);
  for (int i = 0; i < n; ++i)
    for (int k = rp[i]; k < rp[i + 1]; ++k)
      if (ci[k] == i) diag[i] = k;
  const int np = S.ksteps + rpl;
  constexpr int kPadStep = -1, kNone = -2;  // a padding step; no terms
  std::vector<int> posq((size_t)np * lanes);  // position of (p, l), or kPadStep / kNone
  for (int l = 0; l < lanes; ++l) {
    for (int st = 0; st < S.ksteps; ++st) {
      const int32_t e = S.ent[(size_t)st * lanes + l];
      posq[(size_t)st * lanes + l] = (e & bcs::kEntPad) ? kPadStep : (e & bcs::kEntPosMask);
    }
    for (int j = 0; j < rpl; ++j) {
      const int rj = S.row[(size_t)j * lanes + l];
      posq[(size_t)(S.ksteps + j) * lanes + l] = (rj >= 0 && rj < n) ? (diag[rj] & bcs::kEntPosMask) : kNone;
    }
  }
  const int32_t* jofs = m.htab.data() + m.jofs_at;
  const int32_t* jterm = m.htab.data() + m.jterm_at;
  auto count = [&](int q) { return q == kPadStep ? 1 : q == kNone ? 0 : jofs[q + 1] - jofs[q]; };
  terms->assign(1 + np, 0);
  (*terms)[0] = jofs[1] - jofs[0];
  for (int p = 0; p < np; ++p)
    for (int l = 0; l < lanes; ++l) (*terms)[1 + p] = std::max((*terms)[1 + p], count(posq[(size_t)p * lanes + l]));
  prog->clear();
  const uint32_t one = (uint32_t)(n + 1) * 8u;
  const uint32_t pad_word = (uint32_t)(mtbase + m.R) * 8u | one << 16;                  // k = 0, y factor 1
  const uint32_t keep_word = (uint32_t)(mtbase + m.R + 1) * 8u | (uint32_t)(n + 2) * 8u << 16;  // 1 x kept value
  auto push = [&](uint32_t w0, double sf) {
    uint64_t sbits;
    std::memcpy(&sbits, &sf, sizeof(sbits));
    prog->push_back((int32_t)w0);
    prog->push_back((int32_t)(uint32_t)(sbits >> 32));  // the low word of a small integer is 0
  };
  auto push_term = [&](int k) {
    const uint32_t w1 = (uint32_t)jterm[2 * k + 1];
    const uint32_t other = w1 & 0xffffu;
    push((uint32_t)(mtbase + jterm[2 * k]) * 8u | (w1 >> 24 ? 1u : 0u) |
             (other == (uint32_t)bcs::kNoSpecies ? one : other * 8u) << 16,
         (double)((int)((w1 >> 16) & 0xffu) - 128));
  };
  for (int t = 0; t < (*terms)[0]; ++t)
    for (int l = 0; l < lanes; ++l) push_term(jofs[0] + t);
  for (int p = 0; p < np; ++p)
    for (int t = 0; t < (*terms)[1 + p]; ++t)
      for (int l = 0; l < lanes; ++l) {
        const int q = posq[(size_t)p * lanes + l];
        if (q == kPadStep && t == 0)
          push(keep_word, 1.0);
        else if (q >= 0 && jofs[q] + t < jofs[q + 1])
          push_term(jofs[q] + t);
        else
          push(pad_word, 0.0);
      }
  return true;
}

// Transposed pattern of (rp, ci): trp/tci its CSR arrays, tpos[q] the CSR
// position in the original matrix of transposed entry q.
void transpose_pattern(int n, const std::vector<int>& rp, const std::vector<int>& ci, std::vector<int>& trp,
                       std::vector<int>& tci, std::vector<int>& tpos) {
  const int nnz = rp[n];
  trp.assign(n + 1, 0);
  tci.assign(nnz, 0);
  tpos.assign(nnz, 0);
  for (int k = 0; k < nnz; ++k) trp[ci[k] + 1]++;
  for (int j = 0; j < n; ++j) trp[j + 1] += trp[j];
  std::vector<int> fill(trp.begin(), trp.end() - 1);
  for (int i = 0; i < n; ++i)
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      const int q = fill[ci[k]]++;
      tci[q] = i;
      tpos[q] = k;
    }
}

// Schedule shapes the specialised kernels may use.  BCS_SCHED overrides the
// mask (tuning).
int sched_allowed(bool /*mixed*/) {
  if (const char* e = std::getenv("BCS_SCHED")) return std::atoi(e) & (bcs::kSchedDiag | bcs::kSchedSpan);
  return bcs::kSchedDiag | bcs::kSchedSpan;
}

// Whether the adjoint kernel of a lanes-per-cell choice fits the LDS (the
// adjoint shares the forward solve's layout, so forward candidates whose
// adjoint would not fit are skipped).
bool adjoint_fits(int n, const std::vector<int>& trp, const std::vector<int>& tci, const std::vector<int>& tpos,
                  int lanes) {
  const int rpl = (n + lanes - 1) / lanes;
  const HostSchedule T = build_schedule_jit(n, trp, tci, tpos, lanes, rpl, sched_allowed(false));
  return T.ksteps > 0 && jit_feasible(T.ksteps, rpl) &&
         layout_fits(wg_layout(n, lanes, rpl, T.ksteps, 1, false, bcs::kWavesPerWg, (int)tci.size()));
}

// ---- ILU(0) preconditioning (kernel body in bcs_ilu.h) ----

// Jacobi sweeps per triangular solve when the options leave the choice to
// the library.
constexpr int kIluSweepsDefault = 3;

// The strict lower (part 0) or strict upper (part 1) triangle of a pattern
// as a CSR pattern of its own; tpos[q] is the position of its entry q in the
// full pattern.
void triangle_pattern(int n, const std::vector<int>& rp, const std::vector<int>& ci, int part,
                      std::vector<int>& trp, std::vector<int>& tci, std::vector<int>& tpos) {
  trp.assign(n + 1, 0);
  tci.clear();
  tpos.clear();
  for (int i = 0; i < n; ++i) {
    for (int k = rp[i]; k < rp[i + 1]; ++k)
      if (part == 0 ? ci[k] < i : ci[k] > i) {
        tci.push_back(ci[k]);
        tpos.push_back(k);
      }
    trp[i + 1] = (int)tci.size();
  }
}

// Gather schedule of a triangle, its rows dealt by their own lengths (the
// spanning shape allowed; a triangle holds no diagonal), with value
// positions in the full pattern.  ksteps = -1 if the schedule's own check
// fails.
HostSchedule triangle_schedule(int n, const std::vector<int>& rp, const std::vector<int>& ci, int part, int lanes) {
  std::vector<int> trp, tci, tpos;
  triangle_pattern(n, rp, ci, part, trp, tci, tpos);
  std::vector<int> ident(tci.size());
  for (size_t q = 0; q < ident.size(); ++q) ident[q] = (int)q;
  const int rpl = (n + lanes - 1) / lanes;
  HostSchedule S = build_schedule_jit(n, trp, tci, ident, lanes, rpl, sched_allowed(false) & bcs::kSchedSpan);
  if (S.ksteps < 0) return S;
  for (int32_t& e : S.ent)
    if (!(e & bcs::kEntPad)) e = tpos[e & bcs::kEntPosMask] | (e & ~bcs::kEntPosMask);
  return S;
}

// The numeric factorisation as a program (format in bcs_ilu.h: FactProg).
// Entry (i, j) of the pattern becomes a_ij - sum_k l_ik u_kj over the
// k < min(i, j) with (i, k) and (k, j) in the pattern (increasing k), divided
// by u_jj when i > j: the IKJ elimination of ILU(0) (Saad, Algorithm 10.4)
// written per entry.  An entry is an operation if it has terms or lies below
// the diagonal (upper entries without terms keep a_ij).  Its level is one
// more than the highest level among its inputs (l_ik, u_kj and the pivot
// u_jj; unchanged entries have level 0), so that the operations of a level
// only read final values; CSR order is a topological order of these
// dependencies.  Each level becomes steps of at most `lanes` operations,
// sorted by term count so that a step's width (its largest term count) pads
// little.  Every row must hold its diagonal.  Returns false if a position
// does not fit 16 bits.
struct IluProgram {
  std::vector<int> widths;      // terms per step
  std::vector<uint32_t> words;  // per step: lanes head words, then widths[st] x lanes term words
};

bool build_ilu_program(int n, const std::vector<int>& rp, const std::vector<int>& ci, int lanes, IluProgram* out) {
  const int nnz = rp[n];
  if (nnz + bcs::kIluSpare > 65536) return false;
  const uint32_t zero = (uint32_t)(nnz + bcs::kIluZero), unit = (uint32_t)(nnz + bcs::kIluUnit),
                 junk = (uint32_t)(nnz + bcs::kIluJunk);
  std::vector<int> at((size_t)n * n, -1), diag(n, -1);
  for (int i = 0; i < n; ++i)
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      at[(size_t)i * n + ci[k]] = k;
      if (ci[k] == i) diag[i] = k;
    }
  struct Op {
    uint32_t head;
    std::vector<uint32_t> terms;
  };
  std::vector<int> level(nnz, 0);
  std::vector<std::vector<Op>> by_level;
  for (int i = 0; i < n; ++i)
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      const int j = ci[k];
      Op op;
      int lv = 0;
      for (int q = rp[i]; q < rp[i + 1] && ci[q] < std::min(i, j); ++q) {
        const int u = at[(size_t)ci[q] * n + j];
        if (u < 0) continue;
        op.terms.push_back((uint32_t)q | ((uint32_t)u << 16));
        lv = std::max(lv, std::max(level[q], level[u]));
      }
      if (i > j)
        lv = std::max(lv, level[diag[j]]);
      else if (op.terms.empty())
        continue;
      op.head = (uint32_t)k | ((uint32_t)(i > j ? diag[j] : (int)unit) << 16);
      level[k] = lv + 1;
      if ((int)by_level.size() < lv + 1) by_level.resize(lv + 1);
      by_level[lv].push_back(std::move(op));
    }
  out->widths.clear();
  out->words.clear();
  for (auto& ops : by_level) {
    std::stable_sort(ops.begin(), ops.end(),
                     [](const Op& a, const Op& b) { return a.terms.size() > b.terms.size(); });
    for (size_t c0 = 0; c0 < ops.size(); c0 += (size_t)lanes) {
      const size_t c1 = std::min(ops.size(), c0 + (size_t)lanes);
      const int w = (int)ops[c0].terms.size();
      out->widths.push_back(w);
      for (int l = 0; l < lanes; ++l) out->words.push_back(c0 + l < c1 ? ops[c0 + l].head : (junk | unit << 16));
      for (int q = 0; q < w; ++q)
        for (int l = 0; l < lanes; ++l) {
          const bool real = c0 + l < c1 && q < (int)ops[c0 + l].terms.size();
          out->words.push_back(real ? ops[c0 + l].terms[q] : (zero | zero << 16));
        }
    }
  }
  return true;
}

// Workgroup LDS of the ILU(0) kernel, in doubles: one block per cell slot
// (stride fs: the factor block of nnz values and the three constants while a
// cell is staged, afterwards the operand block of n values and the zero
// spare element; 8 mod 32 doubles apart so that a wave's slots start on
// different banks), then at tbase the 16-bit tables (value positions of A,
// L_s and U_s, each row's diagonal position and the padding row's) and the
// factorisation program.  The gathers' 16-bit addresses reach the first
// 64 KiB, where every operand block must end.
struct IluLayout {
  int fs = 0, tbase = 0;
  size_t bytes = 0, gather_end = 0;
};

IluLayout ilu_layout(int n, int nnz, int lanes, int ka, int kl, int ku, size_t prog_words) {
  IluLayout L;
  const int v = std::max(nnz + bcs::kIluSpare, n + 1);
  const int v8 = ((v + 7) / 8) * 8;
  L.fs = ((v8 + 31) / 32) * 32 + 8;
  const int slots = slots_per_wg(lanes);
  L.tbase = slots * L.fs;
  const size_t ntab = (size_t)(ka + kl + ku) * lanes + n + 1;
  L.bytes = (size_t)L.tbase * 8 + ((ntab + 1) & ~(size_t)1) * 2 + prog_words * 4;
  L.gather_end = ((size_t)(slots - 1) * L.fs + n + 1) * 8;
  return L;
}

// Registers of an ILU(0) layout (values 2 VGPRs a step, addresses one a
// step, ten register vectors and the sweeps' temporaries): larger layouts
// would spill.
bool ilu_feasible(int ka, int kl, int ku, int rpl) { return 3 * (ka + kl + ku) + 26 * rpl <= 300; }

int upload_ilu(const HostSchedule& SL, const HostSchedule& SU, const std::vector<uint16_t>& tab,
               const IluProgram& prog, Kernel* K) {
  auto al = [](size_t v) { return (v + 15) & ~(size_t)15; };
  const size_t o_rl = 0, o_cl = al(o_rl + SL.row.size() * 2), o_ru = al(o_cl + SL.col.size());
  const size_t o_cu = al(o_ru + SU.row.size() * 2), o_tab = al(o_cu + SU.col.size());
  const size_t o_prog = al(o_tab + tab.size() * 2), total = al(o_prog + prog.words.size() * 4) + 16;
  void* buf = nullptr;
  HIP_TRY(hipMalloc(&buf, total));
  K->ibuf = buf;
  char* p = (char*)buf;
  HIP_TRY(hipMemcpy(p + o_rl, SL.row.data(), SL.row.size() * 2, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p + o_cl, SL.col.data(), SL.col.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p + o_ru, SU.row.data(), SU.row.size() * 2, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p + o_cu, SU.col.data(), SU.col.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p + o_tab, tab.data(), tab.size() * 2, hipMemcpyHostToDevice));
  if (!prog.words.empty())
    HIP_TRY(hipMemcpy(p + o_prog, prog.words.data(), prog.words.size() * 4, hipMemcpyHostToDevice));
  auto dev = [](const HostSchedule& S, const char* row, const char* col) {
    bcs::DevSchedule d{};
    d.ent = nullptr;
    d.row = (const int16_t*)row;
    d.col = (const uint8_t*)col;
    d.ksteps = S.ksteps;
    d.rpl = S.rpl;
    d.flush[0] = S.flush[0];
    d.flush[1] = S.flush[1];
    return d;
  };
  K->dL = dev(SL, p + o_rl, p + o_cl);
  K->dU = dev(SU, p + o_ru, p + o_cu);
  K->ilu_tab = (const uint16_t*)(p + o_tab);
  K->fprog = (const uint32_t*)(p + o_prog);
  K->fprog_words = (int)prog.words.size();
  return BCS_OK;
}

// Build the ILU(0) kernel for one lanes-per-cell choice (forward solves;
// every row holds its diagonal).  Returns BCS_ERR_UNSUPPORTED without a
// message when the layout does not fit or spills.
int make_ilu_kernel(int n, const std::vector<int>& rp, const std::vector<int>& ci, int lanes, int sweeps,
                    Kernel* out) {
  const int nnz = rp[n];
  const int rpl = (n + lanes - 1) / lanes;
  std::vector<int> pos(nnz);
  for (int k = 0; k < nnz; ++k) pos[k] = k;
  const HostSchedule SA = build_schedule_jit(n, rp, ci, pos, lanes, rpl, sched_allowed(false));
  const HostSchedule SL = triangle_schedule(n, rp, ci, 0, lanes);
  const HostSchedule SU = triangle_schedule(n, rp, ci, 1, lanes);
  if (SA.ksteps < 0 || SL.ksteps < 0 || SU.ksteps < 0)
    return fail(BCS_ERR_UNSUPPORTED, "internal error: ILU(0) schedule check failed (lanes = %d)", lanes);
  if (!ilu_feasible(SA.ksteps, SL.ksteps, SU.ksteps, rpl)) return BCS_ERR_UNSUPPORTED;
  IluProgram prog;
  if (!build_ilu_program(n, rp, ci, lanes, &prog)) return BCS_ERR_UNSUPPORTED;
  const IluLayout L = ilu_layout(n, nnz, lanes, SA.ksteps, SL.ksteps, SU.ksteps, prog.words.size());
  if (L.gather_end > 65536 || L.bytes > device_max_lds()) return BCS_ERR_UNSUPPORTED;
  Kernel K;
  K.lanes = lanes;
  K.rpl = rpl;
  K.ksteps = SA.ksteps;
  K.seg = SA.seg;
  K.flags = SA.flags;
  K.ilu = true;
  K.sweeps = sweeps;
  K.fs = L.fs;
  K.layout.tbase = L.tbase;
  K.layout.bytes = L.bytes;
  K.lds = L.bytes;
  // three schedules' values and addresses live in registers at once: packed
  // addresses and a shorter gather window keep the kernel within 256 VGPRs
  const int opt = bcs::kSchedPack | bcs::kSchedWin8;
  const int flags[3] = {SA.flags | opt, SL.flags | opt, SU.flags | opt};
  const int* segs[3] = {SA.seg.data(), SL.seg.data(), SU.seg.data()};
  const int rpls[3] = {rpl, rpl, rpl};
  char err[512] = {0};
  // First built for two waves per SIMD (at most 256 VGPRs: the 64-lane body
  // of the benchmark pattern sits at that limit, and the bound keeps it
  // there); a build that spills under the bound is rebuilt without it.
  for (const int waves : {2, 0}) {
    const int rc = bcs::jit_ilu_kernel(lanes, flags, segs, rpls, nnz, prog.widths.data(), (int)prog.widths.size(),
                                       waves, K.lds, &K.jit, err, sizeof(err));
    if (rc != BCS_OK) return fail(rc, "%s", err);
    if (K.jit.scratch == 0) break;
  }
  if (K.jit.scratch > 0) return BCS_ERR_UNSUPPORTED;  // spills: another lane count serves the pattern
  K.max_blocks = K.jit.max_blocks;
  if (const char* e = std::getenv("BCS_BLOCKS_PER_CU")) {
    const int o = std::atoi(e);
    if (o > 0) K.max_blocks = o;
  }
  std::vector<uint16_t> tab;
  auto push = [&](const HostSchedule& S) {
    for (int32_t e : S.ent) tab.push_back((uint16_t)((e & bcs::kEntPad) ? nnz + bcs::kIluZero : (e & bcs::kEntPosMask)));
  };
  push(SA);
  push(SL);
  push(SU);
  for (int i = 0; i < n; ++i) {
    int d = 0;
    for (int k = rp[i]; k < rp[i + 1]; ++k)
      if (ci[k] == i) d = k;
    tab.push_back((uint16_t)d);
  }
  tab.push_back((uint16_t)(nnz + bcs::kIluUnit));
  int r = upload_schedule(SA, &K);
  if (r == BCS_OK) r = upload_ilu(SL, SU, tab, prog, &K);
  if (r != BCS_OK) {
    free_kernel(&K);
    return r;
  }
  if (verbose())
    std::fprintf(stderr,
                 "[bcs] kernel ilu0 lanes=%d rpl=%d steps A/L/U=%d/%d/%d shapes=%d/%d/%d factor steps=%zu "
                 "words=%zu sweeps=%d lds=%zu blocks/CU=%d\n",
                 lanes, rpl, SA.ksteps, SL.ksteps, SU.ksteps, SA.flags, SL.flags, SU.flags, prog.widths.size(),
                 prog.words.size(), sweeps, K.lds, K.max_blocks);
  *out = K;
  return BCS_OK;
}

// Whether forward FP64 kernels are built for three waves per SIMD first
// (BCS_OCCUPANCY=0 turns it off, for comparisons).
bool occupancy_build() {
  const char* e = std::getenv("BCS_OCCUPANCY");
  return !(e && std::atoi(e) == 0);
}

// Build the kernel for one matrix (A or A^T) and one lanes-per-cell choice.
// Returns BCS_ERR_UNSUPPORTED (without message) when nothing fits.
// force_occ (forward FP64 kernels): 0 = the build chain below; 1 or 2 = only
// the first or second three-wave build, kept even if it spills (for the data
// autotuner, which times it against the others).
int make_kernel(int n, const std::vector<int>& rp, const std::vector<int>& ci, const std::vector<int>& pos,
                int lanes, int adjoint, bool use_jit, int waves_per_eu, bool mixed, Kernel* out,
                bool grouped = false, const bcs_mechanism* mech = nullptr, int force_occ = 0,
                int wpw = bcs::kWavesPerWg) {
  const int rpl = (n + lanes - 1) / lanes;
  Kernel K;
  K.lanes = lanes;
  K.adjoint = adjoint;
  HostSchedule S;
  std::vector<int32_t> mprog;  // J term program (kernels that assemble J)
  if (use_jit) {
    S = build_schedule_jit(n, rp, ci, pos, lanes, rpl, sched_allowed(mixed));
    if (S.ksteps < 0) return fail(BCS_ERR_UNSUPPORTED, "internal error: schedule check failed (lanes = %d)", lanes);
    if (!jit_feasible(S.ksteps, rpl)) return BCS_ERR_UNSUPPORTED;
    K.rpl = rpl;
    K.ksteps = S.ksteps;
    char err[512] = {0};
    if (waves_per_eu == 0)
      if (const char* e = std::getenv("BCS_WAVES_PER_EU")) waves_per_eu = std::max(0, std::atoi(e));
    // Builds tried in turn, the first that compiles without spilling is kept.
    // Forward FP64 kernels: three waves per SIMD with the rarely used slot
    // vectors in LDS (kSchedLean) and packed gather addresses, then the same
    // with a gather window of 8, then the default build (all vectors in
    // registers, occupancy set by the compiler).  The mixed form: two waves
    // per SIMD, then the default build.
    struct Attempt {
      int extra, waves;
    };
    std::vector<Attempt> tries;
    const bool tuned = waves_per_eu == 0 && occupancy_build();
    const Attempt occ_builds[2] = {{bcs::kSchedLean | bcs::kSchedPack, 3},
                                   {bcs::kSchedLean | bcs::kSchedPack | bcs::kSchedWin8, 3}};
    if (force_occ > 0 && !mixed && !adjoint && !grouped) {
      tries.push_back(occ_builds[force_occ - 1]);
    } else {
      if (tuned && !mixed && !adjoint && !grouped) {
        tries.push_back(occ_builds[0]);
        tries.push_back(occ_builds[1]);
      } else if (tuned && mixed) {
        tries.push_back({0, 2});
      }
      tries.push_back({0, waves_per_eu});
    }
    size_t at = 0;
    for (;; ++at) {
      const Attempt& A = tries[at];
      const bool last = at + 1 == tries.size();
      const bool lean = (A.extra & bcs::kSchedLean) != 0;
      K.layout = wg_layout(n, lanes, rpl, S.ksteps, adjoint, lean, wpw, rp[n]);
      if (!layout_fits(K.layout)) {
        if (last) return BCS_ERR_UNSUPPORTED;
        if (verbose())
          std::fprintf(stderr, "[bcs] lanes=%d: build %zu needs %zu bytes of LDS; next build\n", lanes, at,
                       K.layout.bytes);
        continue;
      }
      K.lds = K.layout.bytes;
      if (mech) {
        // after the schedule tables: room for the shared rate constants and
        // the kernel's J term program
        K.mtbase = (int)(K.layout.tbase + table_doubles(n, lanes, S.ksteps));
        const bool fits = mech_program(S, n, lanes, rpl, rp, ci, *mech, K.mtbase, &K.mterms, &mprog);
        K.mwords = (int)mprog.size();
        K.lds = ((size_t)K.mtbase + mech->R + 2 + mprog.size() / 2) * sizeof(double);
        if (!fits || K.lds > device_lds_limit()) {
          if (last) return BCS_ERR_UNSUPPORTED;
          continue;
        }
      }
      const int rc = bcs::jit_kernel(mixed ? "mixed_body" : "fp64_body", adjoint, grouped ? 1 : 0, lanes,
                                     S.flags | A.extra, S.seg.data(), rpl, A.waves, K.lds, &K.jit, err, sizeof(err),
                                     mech ? &K.mterms : nullptr, wpw);
      if (rc != BCS_OK) return fail(rc, "%s", err);
      if (!last && K.jit.scratch > 0) {
        if (verbose())
          std::fprintf(stderr, "[bcs] lanes=%d: build %zu spills %d bytes per lane; next build\n", lanes, at,
                       K.jit.scratch);
        continue;
      }
      break;
    }
    K.occ = !tries[at].extra ? false : true;
    K.occ_flags = tries[at].extra;
    K.waves = tries[at].waves;
    K.wpw = wpw;
    // a forward candidate that spills registers is dropped (another lane
    // count serves the pattern); the adjoint and the mixed form keep theirs
    if (K.jit.scratch > 0 && !adjoint && !mixed && force_occ == 0) return BCS_ERR_UNSUPPORTED;
    K.max_blocks = K.jit.max_blocks;
    K.seg = S.seg;
    K.flags = S.flags;
  } else {
    if (mixed) return BCS_ERR_UNSUPPORTED;  // the mixed form exists only as specialised kernels
    if (wpw != bcs::kWavesPerWg) return BCS_ERR_UNSUPPORTED;  // precompiled with the default workgroup
    int nv = 0;
    const bcs::Variant* vs = all_variants(&nv);
    const bcs::Variant* best = nullptr;
    for (int q = 0; q < nv; ++q) {
      const bcs::Variant& v = vs[q];
      if (v.lanes != lanes || v.rpl < rpl) continue;
      HostSchedule T = build_schedule(n, rp, ci, pos, lanes, v.rpl, v.kmax);
      if (T.ksteps > v.kmax ||
          !layout_fits(wg_layout(n, lanes, v.rpl, v.kmax, adjoint, false, bcs::kWavesPerWg, rp[n])))
        continue;
      if (!best || v.rpl < best->rpl || (v.rpl == best->rpl && v.kmax < best->kmax)) {
        best = &v;
        S = std::move(T);
      }
    }
    if (!best) return BCS_ERR_UNSUPPORTED;
    K.var = best;
    K.rpl = best->rpl;
    K.ksteps = best->kmax;
    K.layout = wg_layout(n, lanes, best->rpl, best->kmax, adjoint, false, bcs::kWavesPerWg, rp[n]);
    K.lds = K.layout.bytes;
    int nb = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, best->fp64_kernel, bcs::kWgThreads, K.lds));
    K.max_blocks = std::max(nb, 1);
  }
  // tuning override: resident workgroups per CU assumed when sizing the grid
  if (const char* e = std::getenv("BCS_BLOCKS_PER_CU")) {
    const int o = std::atoi(e);
    if (o > 0) K.max_blocks = o;
  }
  const int rc = upload_schedule(S, &K);
  if (rc != BCS_OK) {
    free_kernel(&K);
    return rc;
  }
  if (!mprog.empty()) {
    hipError_t e = hipMalloc(&K.mbuf, mprog.size() * sizeof(int32_t));
    if (e == hipSuccess) e = hipMemcpy(K.mbuf, mprog.data(), mprog.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      free_kernel(&K);
      return fail(BCS_ERR_HIP, "J term program: %s", hipGetErrorString(e));
    }
  }
  if (verbose())
    std::fprintf(stderr,
                 "[bcs] kernel %s%s lanes=%d rpl=%d steps=%d shape=%d extra=%d waves=%d adjoint=%d lds=%zu "
                 "blocks/CU=%d\n",
                 use_jit ? "jit" : "precompiled", mixed ? " mixed" : "", lanes, K.rpl, K.ksteps, K.flags, K.occ_flags,
                 K.waves, adjoint, K.lds, K.max_blocks);
  *out = K;
  return BCS_OK;
}

}  // namespace

namespace {

// Validate a CSR pattern: row_ptr[0] = 0, row_ptr[n] = nnz, non-decreasing
// row_ptr, strictly increasing columns in [0, n) per row, the diagonal in
// every row if need_diag, and n within the kernels' 255 rows (8-bit gather
// indices, with index n the zero spare element).
int check_pattern(int32_t n, int32_t nnz, const int32_t* row_ptr, const int32_t* col_idx, bool need_diag) {
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
  if (need_diag)
    for (int i = 0; i < n; ++i)
      if (diag[i] < 0) return fail(BCS_ERR_PATTERN, "row %d has no diagonal entry", i);
  if (n > 255) return fail(BCS_ERR_UNSUPPORTED, "n = %d exceeds the supported 255 rows per cell", n);
  return BCS_OK;
}

}  // namespace

struct bcs_plan {
  int n = 0, nnz = 0;
  int device = 0;
  int num_cu = 0;
  bcs_options opt{};
  std::vector<int> rp, ci;
  Kernel fwd, adj;
  const bcs_mechanism* mech = nullptr;  // plans made by bcs_plan_create_mech
  Kernel fwd_mech;                      // their forward kernel that assembles J while staging
  int32_t* diag_pos = nullptr;
  int16_t* coo_row = nullptr;
  int16_t* coo_col = nullptr;
};

// Scratch of bcs_solve_batch_noalloc: the contents of a caller's workspace
// (work queue, cost-order sort state, the order itself) in a library-owned
// device array, one copy on every GPU the library runs on, held until the
// process ends.  In host code the array's name is only a host-side stand-in:
// host code uses the device address hipGetSymbolAddress returns for each
// device (scratch_address), never the name itself.
static __device__ __align__(256) unsigned char scratch[BCS_NOALLOC_MAX_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Resolve this device's copy of `scratch` (the current device; once per
// device, at plan creation).
int scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(BCS_ERR_UNSUPPORTED, "device index %d >= %d", device, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_addr[device]) return BCS_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(BCS_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
  g_scratch_addr[device] = ptr;
  return BCS_OK;
}

void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_addr[device];
}

}  // namespace

namespace {

void release(bcs_plan* p) {
  if (!p) return;
  int cur = 0;
  if (hipGetDevice(&cur) == hipSuccess && cur != p->device) (void)hipSetDevice(p->device);
  free_kernel(&p->fwd);
  free_kernel(&p->adj);
  free_kernel(&p->fwd_mech);
  if (p->diag_pos) (void)hipFree(p->diag_pos);
  if (p->coo_row) (void)hipFree(p->coo_row);
  if (cur != p->device) (void)hipSetDevice(cur);
  delete p;
}

bcs::KParams base_params(const bcs_plan* p, int64_t ncells, const double* values, const double* gamma,
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
  P.visits = g_visits;
  P.precond = p->opt.precond;
  P.kind = p->opt.matrix_kind;
  P.rr = p->opt.residual_replacement;
  P.brs = p->opt.breakdown_restarts;
  P.inner_rtol = p->opt.inner_rtol;
  P.max_refine = p->opt.max_refine;
  P.budget = p->opt.refine_budget == BCS_BUDGET_CELL ? 1 : 0;
  P.diag_pos = p->diag_pos;
  P.coo_row = p->coo_row;
  P.coo_col = p->coo_col;
  return P;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t ws_bytes(int64_t ncells) {
  return align256((size_t)bcs::kWsOrderOffset + (size_t)std::max<int64_t>(ncells, 0) * sizeof(int32_t));
}

// Prologue of a solve on `stream`: point the kernel at its work queue in the
// workspace and clear it, and, with cell_order on, cells solved on their own
// (not shared_scalars), per-cell gamma and more cells than the launch has
// slots (`slots`; 0 = not known), sort the cells by gamma into the
// workspace's order array and point the solve at it.  When every cell has a
// slot of its own from the start, the order cannot even out anything: slot
// k then solves cell k and nothing else (no queue, no claims: P->queue is
// null and nothing is launched here), instead of half of the slots taking
// the cells in pairs.  Block-cells (N) runs keep the queue.  With more cells
// than slots (and `slots` known) and a kernel built with the path
// (`first_claims`), the slots' first claims are handed out without the
// counter (slot k takes the positions from k * cells per claim) and the
// counter starts past them, so the launch does not open with every slot's
// atomic on one address at once.
int prologue(const bcs_plan* p, bcs::KParams* P, void* ws, hipStream_t stream, int64_t slots, bool first_claims) {
  char* w = (char*)ws;
  P->order = nullptr;
  P->qfirst = 0;
  if (slots > 0 && P->ncells <= slots && p->opt.shared_scalars == 0) {
    P->queue = nullptr;
    return BCS_OK;
  }
  P->queue = (unsigned long long*)w;
  const bool use_order = p->opt.cell_order == 1 && p->opt.shared_scalars == 0 && p->opt.matrix_kind == BCS_J_GAMMA &&
                         P->gamma_stride != 0 && P->ncells >= 2 && P->ncells <= INT32_MAX;
  int32_t* order = use_order ? (int32_t*)(w + bcs::kWsOrderOffset) : nullptr;
  if (first_claims && slots > 0 && p->opt.shared_scalars == 0)
    P->qfirst = slots * (use_order ? bcs::kClaimGroup : 1);
  const hipError_t e = bcs::launch_solve_prologue(P->queue, (unsigned long long)P->qfirst, P->gamma,
                                                  P->gamma_stride, P->ncells, (uint32_t*)(w + bcs::kWsStateOffset),
                                                  order, stream);
  if (e != hipSuccess) return fail(BCS_ERR_HIP, "solve prologue launch: %s", hipGetErrorString(e));
  P->order = order;
  return BCS_OK;
}

int check_workspace(const bcs_plan* p, int64_t ncells, void* ws, size_t bytes) {
  (void)p;
  if (!ws) return fail(BCS_ERR_ARG, "workspace is NULL");
  if (((uintptr_t)ws & 255u) != 0) return fail(BCS_ERR_ARG, "workspace must be 256-byte aligned");
  if (bytes < ws_bytes(ncells))
    return fail(BCS_ERR_ARG, "workspace of %zu bytes is smaller than the %zu bytes needed for %lld cells", bytes,
                ws_bytes(ncells), (long long)ncells);
  return BCS_OK;
}

// A device workspace owned by the autotuners (they may allocate).
struct OwnedWorkspace {
  void* ptr = nullptr;
  ~OwnedWorkspace() {
    if (ptr) (void)hipFree(ptr);
  }
  int alloc(size_t bytes) {
    if (hipMalloc(&ptr, bytes) != hipSuccess) {
      ptr = nullptr;
      return fail(BCS_ERR_HIP, "autotune: workspace allocation of %zu bytes failed", bytes);
    }
    return BCS_OK;
  }
};

int grid_for(const bcs_plan* p, const Kernel& K, int64_t ncells) {
  const int64_t cells_per_wg = (int64_t)K.wpw * (64 / K.lanes);
  const int64_t need = (ncells + cells_per_wg - 1) / cells_per_wg;
  const int64_t cap = (int64_t)K.max_blocks * p->num_cu;
  return (int)std::max<int64_t>(1, std::min(need, cap));
}

// Whether kernel K's slots take their first claims without the counter (the
// FP64 kernels; the mixed kernel is built without that path: with it, its
// code got slower).
bool first_claims(const bcs_plan* p, const Kernel& K) {
  (void)K;
  return p->opt.precision == BCS_FP64;
}

// Cell slots of a launch of kernel K over ncells cells.
int64_t slots_for(const bcs_plan* p, const Kernel& K, int64_t ncells) {
  return (int64_t)grid_for(p, K, ncells) * K.wpw * (64 / K.lanes);
}

// Fill the launch-specific fields and launch kernel K (forward or adjoint);
// P.queue / P.order come from the prologue.
int launch(const bcs_plan* p, const Kernel& K, bcs::KParams P, hipStream_t stream) {
  P.sched = K.d;
  P.adjoint = K.adjoint;
  const WgLayout& L = K.layout;
  P.xs = L.xs;
  P.wxs = L.wxs;
  P.bbase = L.bbase;
  P.bs = L.bs;
  P.wbs = L.wbs;
  P.yoff = L.yoff;
  P.tbase = L.tbase;
  P.coobase = L.coobase;
  P.mtbase = K.mtbase;
  if (K.ilu) {
    P.schedL = K.dL;
    P.schedU = K.dU;
    P.ilu_tab = K.ilu_tab;
    P.fprog = K.fprog;
    P.fprog_words = K.fprog_words;
    P.sweeps = K.sweeps;
    P.fs = K.fs;
  }
  const int grid = grid_for(p, K, P.ncells);
  const hipError_t e = K.launch(P, grid, stream);
  if (e != hipSuccess) return fail(BCS_ERR_HIP, "solve launch: %s", hipGetErrorString(e));
  return BCS_OK;
}

// Time one solve (prologue and launch) with kernel K (forward) on a batch
// already on the device, with workspace ws: a warm-up solve, then the best of
// `reps` timed solves.
int time_launches(const bcs_plan* p, const Kernel& K, const bcs::KParams& P0, void* ws, int reps, double* seconds) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(BCS_ERR_HIP, "autotune: event creation failed");
  }
  double best = 1e300;
  int rc = BCS_OK;
  for (int rep = 0; rep <= reps && rc == BCS_OK; ++rep) {
    (void)hipEventRecord(e0, nullptr);
    bcs::KParams P = P0;
    rc = prologue(p, &P, ws, nullptr, slots_for(p, K, P.ncells), first_claims(p, K));
    if (rc == BCS_OK) rc = launch(p, K, P, nullptr);
    (void)hipEventRecord(e1, nullptr);
    if (rc != BCS_OK) break;
    if (hipEventSynchronize(e1) != hipSuccess) {
      rc = fail(BCS_ERR_HIP, "autotune launch failed");
      break;
    }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (rep > 0) best = std::min(best, (double)ms * 1e-3);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *seconds = best;
  return rc;
}

// Time kernel K on a synthetic batch of the plan's pattern.  Cell c has unit
// diagonal and off-diagonal entries s_c * u / (row length), u uniform in
// [-1, 1] and s_c uniform in [0, 0.95): row diagonally dominant, with a
// spread of conditioning so that cells need widely different iteration
// counts at rtol 1e-10 -- the regime in which slots refill at different
// times.  Returns seconds per launch.
int time_kernel_synthetic(const bcs_plan* p, const Kernel& K, double* seconds) {
  const int64_t C = (int64_t)std::max(8192, 96 * p->num_cu);
  const int n = p->n, nnz = p->nnz;
  std::vector<double> hv((size_t)C * nnz), hb((size_t)C * n);
  uint64_t s = 0x9E3779B97F4A7C15ull;
  auto rnd = [&s]() {  // splitmix64 -> [0, 1)
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
  };
  for (int64_t c = 0; c < C; ++c) {
    const double sc = 0.95 * rnd();
    for (int i = 0; i < n; ++i) {
      const int len = std::max(1, p->rp[i + 1] - p->rp[i] - 1);
      for (int k = p->rp[i]; k < p->rp[i + 1]; ++k)
        hv[(size_t)c * nnz + k] = (p->ci[k] == i) ? 1.0 : sc * (2.0 * rnd() - 1.0) / len;
    }
    for (int i = 0; i < n; ++i) hb[(size_t)c * n + i] = rnd() - 0.5;
  }
  double *dv = nullptr, *db = nullptr, *dg = nullptr, *dx = nullptr, *dr = nullptr;
  int32_t *di = nullptr, *ds = nullptr;
  auto cleanup = [&]() {
    for (void* q : {(void*)dv, (void*)db, (void*)dg, (void*)dx, (void*)dr, (void*)di, (void*)ds})
      if (q) (void)hipFree(q);
  };
  hipError_t e = hipMalloc((void**)&dv, hv.size() * 8);
  if (e == hipSuccess) e = hipMalloc((void**)&db, hb.size() * 8);
  if (e == hipSuccess) e = hipMalloc((void**)&dg, 8);
  if (e == hipSuccess) e = hipMalloc((void**)&dx, hb.size() * 8);
  if (e == hipSuccess) e = hipMalloc((void**)&dr, C * 8);
  if (e == hipSuccess) e = hipMalloc((void**)&di, C * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&ds, C * 4);
  if (e == hipSuccess) e = hipMemcpy(dv, hv.data(), hv.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(db, hb.data(), hb.size() * 8, hipMemcpyHostToDevice);
  const double g0 = 0.0;
  if (e == hipSuccess) e = hipMemcpy(dg, &g0, 8, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    cleanup();
    return fail(BCS_ERR_HIP, "autotune setup: %s", hipGetErrorString(e));
  }
  bcs::KParams P = base_params(p, C, dv, dg, 0, 1e-10, 200);
  P.visits = nullptr;
  P.kind = bcs::kADirect;
  P.b = db;
  P.xin = dx;
  P.x = dx;
  P.iters = di;
  P.resid = dr;
  P.status = ds;
  P.grad_vals = nullptr;
  P.x0 = nullptr;
  OwnedWorkspace ws;
  int rc = ws.alloc(ws_bytes(C));
  if (rc == BCS_OK) rc = time_launches(p, K, P, ws.ptr, 2, seconds);
  cleanup();
  return rc;
}

}  // namespace

namespace {

// A mechanism plan's forward kernel that assembles J while staging, built for
// the lane count of the plan's forward kernel (again whenever a tuner changes it).
int sync_mech(bcs_plan* p) {
  if (!p->mech || (p->fwd_mech.buf && p->fwd_mech.lanes == p->fwd.lanes)) return BCS_OK;
  std::vector<int> pos(p->nnz);
  for (int k = 0; k < p->nnz; ++k) pos[k] = k;
  Kernel K;
  g_err.clear();
  const int rc = make_kernel(p->n, p->rp, p->ci, pos, p->fwd.lanes, 0, true, 0, false, &K, false, p->mech);
  if (rc != BCS_OK)
    return g_err.empty() ? fail(rc, "no layout holds the mechanism kernel at %d lanes per cell (LDS)", p->fwd.lanes)
                         : rc;
  free_kernel(&p->fwd_mech);
  p->fwd_mech = K;
  return BCS_OK;
}

}  // namespace

namespace bcs {
int set_error(int code, const char* msg) { return fail(code, "%s", msg); }
void clear_error() { g_err.clear(); }
}  // namespace bcs

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
  o->jit = 1;
  o->autotune = 1;
  o->cell_order = 1;
  o->shared_scalars = 0;
  o->refine_budget = BCS_BUDGET_INNER;
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
  if (!row_ptr || !col_idx) return fail(BCS_ERR_ARG, "row_ptr/col_idx is NULL");
  if (o.precision != BCS_FP64 && o.precision != BCS_FP32_REFINE)
    return fail(BCS_ERR_ARG, "unknown precision %d", o.precision);
  if (o.precond != BCS_PRECOND_NONE && o.precond != BCS_PRECOND_JACOBI && o.precond != BCS_PRECOND_ILU0)
    return fail(BCS_ERR_ARG, "unknown preconditioner %d", o.precond);
  const bool ilu = o.precond == BCS_PRECOND_ILU0;
  if (ilu && (o.precision != BCS_FP64 || o.jit != 1 || o.shared_scalars != 0))
    return fail(BCS_ERR_ARG, "BCS_PRECOND_ILU0 needs FP64, jit = 1 and shared_scalars = 0");
  if (o.ilu_sweeps < 0 || o.ilu_sweeps > 16 || (!ilu && o.ilu_sweeps != 0))
    return fail(BCS_ERR_ARG, "ilu_sweeps must be in [0, 16], and 0 unless precond is BCS_PRECOND_ILU0");
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
  if (o.jit != 0 && o.jit != 1) return fail(BCS_ERR_ARG, "jit must be 0 or 1");
  if (o.autotune != 0 && o.autotune != 1) return fail(BCS_ERR_ARG, "autotune must be 0 or 1");
  if (o.cell_order != 0 && o.cell_order != 1) return fail(BCS_ERR_ARG, "cell_order must be 0 or 1");
  if (o.shared_scalars != 0 && o.shared_scalars != 1) return fail(BCS_ERR_ARG, "shared_scalars must be 0 or 1");
  if (o.shared_scalars == 1 && (o.precision != BCS_FP64 || o.jit != 1 || o.lanes_per_cell == 0))
    return fail(BCS_ERR_ARG, "shared_scalars needs FP64, jit = 1 and lanes_per_cell 16, 32 or 64");
  if (o.refine_budget != BCS_BUDGET_INNER && o.refine_budget != BCS_BUDGET_CELL)
    return fail(BCS_ERR_ARG, "refine_budget must be BCS_BUDGET_INNER or BCS_BUDGET_CELL");
  if (o.waves_per_group != 0 && o.waves_per_group != 1 && o.waves_per_group != 2 && o.waves_per_group != 4 &&
      o.waves_per_group != 8)
    return fail(BCS_ERR_ARG, "waves_per_group must be 0, 1, 2, 4 or 8 (got %d)", o.waves_per_group);
  if (o.waves_per_group != 0 && (o.jit != 1 || o.precision != BCS_FP64 || o.precond == BCS_PRECOND_ILU0 ||
                                 o.shared_scalars == 1))
    return fail(BCS_ERR_UNSUPPORTED, "waves_per_group needs jit = 1, FP64, no ILU0 and shared_scalars = 0");

  const bool need_diag = o.matrix_kind == BCS_J_GAMMA || o.precond == BCS_PRECOND_JACOBI || ilu ||
                         o.precision == BCS_FP32_REFINE;
  const int prc = check_pattern(n, nnz, row_ptr, col_idx, need_diag);
  if (prc != BCS_OK) return prc;

  if (ilu && o.ilu_sweeps == 0) o.ilu_sweeps = kIluSweepsDefault;
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
  {
    const int src = scratch_init(p->device);  // the no-allocation entry point's scratch on this device
    if (src != BCS_OK) {
      delete p;
      return src;
    }
  }

  // device tables shared by every kernel of the plan
  std::vector<int16_t> crow(nnz), ccol(nnz);
  std::vector<int> diag(n, 0);  // an absent diagonal (allowed without Jacobi) is never read: 0 keeps it in bounds
  for (int i = 0; i < n; ++i)
    for (int k = p->rp[i]; k < p->rp[i + 1]; ++k) {
      crow[k] = (int16_t)i;
      ccol[k] = (int16_t)p->ci[k];
      if (p->ci[k] == i) diag[i] = k;
    }
  hipError_t e = hipMalloc((void**)&p->diag_pos, sizeof(int32_t) * n);
  if (e == hipSuccess) e = hipMemcpy(p->diag_pos, diag.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc((void**)&p->coo_row, sizeof(int16_t) * 2 * nnz);
  if (e == hipSuccess) {
    p->coo_col = p->coo_row + nnz;
    e = hipMemcpy(p->coo_row, crow.data(), sizeof(int16_t) * nnz, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMemcpy(p->coo_col, ccol.data(), sizeof(int16_t) * nnz, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    release(p);
    return fail(BCS_ERR_HIP, "plan allocation: %s", hipGetErrorString(e));
  }

  // A and A^T patterns with value positions
  std::vector<int> pos(nnz);
  for (int k = 0; k < nnz; ++k) pos[k] = k;
  std::vector<int> trp, tci, tpos;
  transpose_pattern(n, p->rp, p->ci, trp, tci, tpos);

  // Lanes per cell.  Candidates that fit are either timed on a synthetic
  // batch (autotune) or ranked by wave-steps per cell (ksteps * lanes / 64).
  const bool jit = o.jit == 1;
  const bool mixed = o.precision == BCS_FP32_REFINE;
  if (mixed && !jit) {
    release(p);
    return fail(BCS_ERR_UNSUPPORTED, "FP32_REFINE needs jit = 1 (its kernels are compiled per pattern)");
  }
  Kernel best;
  double best_cost = 1e300;
  int rc = BCS_OK;
  const int cand[3] = {16, 32, 64};
  for (int L : cand) {
    if (o.lanes_per_cell != 0 && o.lanes_per_cell != L) continue;
    if (!ilu && !adjoint_fits(n, trp, tci, tpos, L)) continue;
    Kernel K;
    g_err.clear();
    int r = ilu ? make_ilu_kernel(n, p->rp, p->ci, L, o.ilu_sweeps, &K)
                : make_kernel(n, p->rp, p->ci, pos, L, 0, jit, 0, mixed, &K, o.shared_scalars == 1, nullptr, 0,
                              o.waves_per_group ? o.waves_per_group : bcs::kWavesPerWg);
    if (r == BCS_ERR_UNSUPPORTED && g_err.empty()) continue;
    if (r != BCS_OK) {
      rc = r;
      break;
    }
    double cost = (double)K.ksteps * L / 64.0;
    if (o.autotune == 1 && o.lanes_per_cell == 0) {
      r = time_kernel_synthetic(p, K, &cost);
      if (r != BCS_OK) {
        free_kernel(&K);
        rc = r;
        break;
      }
      if (verbose()) std::fprintf(stderr, "[bcs] autotune lanes=%d: %.1f us per launch\n", L, cost * 1e6);
    }
    if (cost < best_cost) {
      free_kernel(&best);
      best = K;
      best_cost = cost;
    } else {
      free_kernel(&K);
    }
  }
  if (rc == BCS_OK && !best.buf)
    rc = fail(BCS_ERR_UNSUPPORTED, "no kernel layout holds this pattern (n = %d, nnz = %d)", n, nnz);
  if (rc == BCS_OK) {
    p->fwd = best;
    g_err.clear();
    if (!ilu) {  // ILU(0) plans solve forward systems only
      rc = make_kernel(n, trp, tci, tpos, best.lanes, 1, jit, 0, false, &p->adj);
      if (rc == BCS_ERR_UNSUPPORTED && g_err.empty())
        rc = fail(BCS_ERR_UNSUPPORTED, "no kernel layout holds the transposed pattern");
    }
  } else {
    free_kernel(&best);
  }
  if (rc != BCS_OK) {
    release(p);
    return rc;
  }
  *out = p;
  return BCS_OK;
}

void bcs_plan_destroy(bcs_plan* plan) { release(plan); }

int bcs_plan_autotune(bcs_plan* p, int64_t ncells, const double* values, const double* gamma,
                      int64_t gamma_stride, const double* b, double rtol, int32_t maxit, double* x,
                      int32_t* iters, double* resid, int32_t* status, int32_t* lanes_out) {
  g_err.clear();
  if (!p) return fail(BCS_ERR_ARG, "plan is NULL");
  if (ncells <= 0) return fail(BCS_ERR_ARG, "autotune needs ncells > 0");
  if (p->opt.shared_scalars == 1)
    return fail(BCS_ERR_UNSUPPORTED, "a shared_scalars plan has a fixed lanes_per_cell; nothing to tune");
  if (!values || !b || !x || !iters || !resid || !status || (p->opt.matrix_kind == BCS_J_GAMMA && !gamma))
    return fail(BCS_ERR_ARG, "values/gamma/b/x/iters/resid/status is NULL");
  if (!(rtol > 0.0) || maxit < 1) return fail(BCS_ERR_ARG, "bad rtol/maxit");
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess || cur != p->device)
    return fail(BCS_ERR_ARG, "the plan belongs to device %d, current device is %d", p->device, cur);
  if (hipDeviceSynchronize() != hipSuccess) return fail(BCS_ERR_HIP, "device synchronisation failed");
  bcs::KParams P = base_params(p, ncells, values, gamma, gamma_stride, rtol, maxit);
  P.b = b;
  P.x = x;
  P.iters = iters;
  P.resid = resid;
  P.status = status;
  P.refinements = nullptr;
  P.x0 = nullptr;
  std::vector<int> pos(p->nnz);
  for (int k = 0; k < p->nnz; ++k) pos[k] = k;
  const bool jit = p->opt.jit == 1;
  std::vector<int> trp, tci, tpos;
  transpose_pattern(p->n, p->rp, p->ci, trp, tci, tpos);
  OwnedWorkspace ws;
  int rc = ws.alloc(ws_bytes(ncells));
  if (rc != BCS_OK) return rc;
  const bool ilu = p->opt.precond == BCS_PRECOND_ILU0;
  const int cand[3] = {16, 32, 64};
  // Candidates: the plan's kernel (index 0), every lane count's kernel from
  // the build chain, and for forward FP64 plans also the three-wave builds
  // the chain dropped because they spill (a few spilled registers can cost
  // less than a wave per SIMD); then, for the winner, other workgroup sizes.
  // Launch times drift (clocks, caches), so the candidates are timed in
  // rounds, each round launching every candidate once, and a challenger
  // must beat the plan's kernel by a margin: 1%, 3% for a spilling build.
  const bool fp64_fwd = !ilu && p->opt.precision == BCS_FP64 && p->opt.shared_scalars == 0 && jit &&
                        occupancy_build();
  struct Cand {
    Kernel K;
    int force = 0;
    double t = 1e300;
  };
  std::vector<Cand> cs;
  cs.push_back({p->fwd, 0, 1e300});
  auto drop_all = [&](size_t keep) {
    for (size_t i = 1; i < cs.size(); ++i)
      if (i != keep) free_kernel(&cs[i].K);
  };
  for (int L : cand) {
    if (!ilu && !adjoint_fits(p->n, trp, tci, tpos, L)) continue;
    for (int force = 0; force <= (fp64_fwd ? 2 : 0); ++force) {
      if (L == p->fwd.lanes && force == 0) continue;  // the plan's own kernel
      Kernel K;
      g_err.clear();
      int r = ilu ? make_ilu_kernel(p->n, p->rp, p->ci, L, p->opt.ilu_sweeps, &K)
                  : make_kernel(p->n, p->rp, p->ci, pos, L, 0, jit, 0, p->opt.precision == BCS_FP32_REFINE, &K,
                                false, nullptr, force, p->fwd.wpw);
      if (r == BCS_ERR_UNSUPPORTED && g_err.empty()) continue;
      if (r != BCS_OK) {
        drop_all(0);
        return r;
      }
      if (force > 0 && K.jit.scratch == 0) {  // the chain keeps such a build itself
        free_kernel(&K);
        continue;
      }
      cs.push_back({K, force, 1e300});
    }
  }
  auto time_rounds = [&](const std::vector<size_t>& idx) -> int {
    for (size_t i : idx) cs[i].t = 1e300;
    for (int round = 0; round < 3; ++round)
      for (size_t i : idx) {
        double t = 0;
        const int r = time_launches(p, cs[i].K, P, ws.ptr, round == 0 ? 2 : 1, &t);
        if (r != BCS_OK) return r;
        cs[i].t = std::min(cs[i].t, t);
      }
    return BCS_OK;
  };
  std::vector<size_t> all(cs.size());
  for (size_t i = 0; i < cs.size(); ++i) all[i] = i;
  rc = time_rounds(all);
  if (rc != BCS_OK) {
    drop_all(0);
    return rc;
  }
  if (verbose())
    for (const Cand& c : cs)
      std::fprintf(stderr, "[bcs] autotune (data) lanes=%d build=%d spill=%d: %.1f us\n", c.K.lanes, c.force,
                   c.K.jit.scratch, c.t * 1e6);
  size_t w = 0;
  for (size_t i = 1; i < cs.size(); ++i) {
    const double margin = cs[i].K.jit.scratch > 0 ? 0.97 : 0.99;
    if (cs[i].t < cs[0].t * margin && cs[i].t < cs[w].t) w = i;
  }
  // waves per workgroup for the winner (the waves share only the schedule
  // copy, so the count sets how often that copy is made and how LDS and
  // registers round into whole workgroups per CU)
  if (fp64_fwd && p->opt.waves_per_group == 0 && !cs[w].K.occ && cs[w].K.var == nullptr &&
      cs[w].K.jit.scratch == 0) {
    const size_t first = cs.size();
    for (int wpw : {2, 8}) {
      if (wpw == cs[w].K.wpw) continue;
      Kernel K;
      g_err.clear();
      int r = make_kernel(p->n, p->rp, p->ci, pos, cs[w].K.lanes, 0, jit, 0, false, &K, false, nullptr, 0, wpw);
      if (r == BCS_ERR_UNSUPPORTED && g_err.empty()) continue;
      if (r != BCS_OK) {
        drop_all(0);
        return r;
      }
      cs.push_back({K, 0, 1e300});
    }
    std::vector<size_t> idx{w};  // the winner, timed again beside the workgroup sizes
    for (size_t i = first; i < cs.size(); ++i) idx.push_back(i);
    rc = time_rounds(idx);
    if (rc != BCS_OK) {
      drop_all(0);
      return rc;
    }
    if (verbose())
      for (size_t i : idx)
        std::fprintf(stderr, "[bcs] autotune (data) lanes=%d waves/workgroup=%d: %.1f us\n", cs[i].K.lanes,
                     cs[i].K.wpw, cs[i].t * 1e6);
    // a workgroup size replaces the winner only if 3% faster (sizes measured
    // within about 1% of each other, with that much noise between runs)
    size_t w2 = w;
    for (size_t i = first; i < cs.size(); ++i)
      if (cs[i].t < cs[w].t * 0.97 && cs[i].t < cs[w2].t) w2 = i;
    w = w2;
  }
  drop_all(w);
  if (w != 0) {
    free_kernel(&p->fwd);
    p->fwd = cs[w].K;
  }
  const int best_lanes = p->fwd.lanes;
  if (!ilu && p->adj.lanes != best_lanes) {
    Kernel A;
    g_err.clear();
    rc = make_kernel(p->n, trp, tci, tpos, best_lanes, 1, jit, 0, false, &A);
    if (rc != BCS_OK) return g_err.empty() ? fail(rc, "no kernel layout holds the transposed pattern") : rc;
    free_kernel(&p->adj);
    p->adj = A;
  }
  rc = sync_mech(p);
  if (rc != BCS_OK) return rc;
  if (lanes_out) *lanes_out = best_lanes;
  return BCS_OK;
}

int bcs_plan_info(const bcs_plan* p, int32_t* lanes, int32_t* rpl, int32_t* steps, int32_t* cells_per_wg) {
  if (!p) return fail(BCS_ERR_ARG, "plan is NULL");
  if (lanes) *lanes = p->fwd.lanes;
  if (rpl) *rpl = p->fwd.rpl;
  if (steps) *steps = p->fwd.ksteps;
  if (cells_per_wg) *cells_per_wg = p->fwd.wpw * (64 / p->fwd.lanes);
  return BCS_OK;
}

static_assert(BCS_SCHED_SPAN == bcs::kSchedSpan && BCS_SCHED_DIAG == bcs::kSchedDiag, "schedule shape bits");

int bcs_schedule_describe(int32_t n, int32_t nnz, const int32_t* row_ptr, const int32_t* col_idx, int32_t lanes,
                          int32_t transpose, int32_t shapes, int32_t* steps, int32_t* rows_per_lane, int32_t* shape,
                          int32_t* seg, int16_t* row, int32_t* pos, uint8_t* col) {
  g_err.clear();
  if (n <= 0 || nnz < 1 || !row_ptr || !col_idx) return fail(BCS_ERR_ARG, "bad pattern arguments");
  if (lanes != 16 && lanes != 32 && lanes != 64) return fail(BCS_ERR_ARG, "lanes must be 16, 32 or 64");
  if (transpose < BCS_PART_A || transpose > BCS_PART_UPPER) return fail(BCS_ERR_ARG, "unknown matrix part %d", transpose);
  if (shapes < 0 || shapes > (BCS_SCHED_SPAN | BCS_SCHED_DIAG)) return fail(BCS_ERR_ARG, "unknown shapes %d", shapes);
  const int prc = check_pattern(n, nnz, row_ptr, col_idx, false);
  if (prc != BCS_OK) return prc;
  std::vector<int> rp(row_ptr, row_ptr + n + 1), ci(col_idx, col_idx + nnz), pos0(nnz);
  for (int k = 0; k < nnz; ++k) pos0[k] = k;
  std::vector<int> trp, tci, tpos;
  if (transpose == BCS_PART_AT) transpose_pattern(n, rp, ci, trp, tci, tpos);
  const int rpl = (n + lanes - 1) / lanes;
  HostSchedule S;
  if (transpose == BCS_PART_LOWER || transpose == BCS_PART_UPPER) {
    std::vector<int> lrp, lci, lpos;
    triangle_pattern(n, rp, ci, transpose == BCS_PART_LOWER ? 0 : 1, lrp, lci, lpos);
    std::vector<int> ident(lci.size());
    for (size_t q = 0; q < ident.size(); ++q) ident[q] = (int)q;
    S = build_schedule_jit(n, lrp, lci, ident, lanes, rpl, shapes & bcs::kSchedSpan);
    if (S.ksteps >= 0)
      for (int32_t& e : S.ent)
        if (!(e & bcs::kEntPad)) e = lpos[e & bcs::kEntPosMask] | (e & ~bcs::kEntPosMask);
  } else {
    S = transpose ? build_schedule_jit(n, trp, tci, tpos, lanes, rpl, shapes)
                  : build_schedule_jit(n, rp, ci, pos0, lanes, rpl, shapes);
  }
  if (S.ksteps < 0) return fail(BCS_ERR_UNSUPPORTED, "internal error: schedule check failed (lanes = %d)", lanes);
  if (steps) *steps = S.ksteps;
  if (rows_per_lane) *rows_per_lane = rpl;
  if (shape) *shape = S.flags;
  if (seg)
    for (int j = 0; j < rpl; ++j) seg[j] = S.seg[j];
  if (row)
    for (size_t q = 0; q < S.row.size(); ++q) row[q] = S.row[q];
  for (size_t q = 0; q < S.ent.size(); ++q) {
    const bool pad = (S.ent[q] & bcs::kEntPad) != 0;
    if (pos) pos[q] = pad ? -1 : (S.ent[q] & bcs::kEntPosMask);
    if (col) col[q] = S.col[q];
  }
  return BCS_OK;
}

int bcs_ilu_describe(int32_t n, int32_t nnz, const int32_t* row_ptr, const int32_t* col_idx, int32_t lanes,
                     int32_t* nsteps, int32_t* widths, int32_t* nwords, uint32_t* words) {
  g_err.clear();
  if (n <= 0 || nnz < 1 || !row_ptr || !col_idx) return fail(BCS_ERR_ARG, "bad pattern arguments");
  if (lanes != 16 && lanes != 32 && lanes != 64) return fail(BCS_ERR_ARG, "lanes must be 16, 32 or 64");
  const int prc = check_pattern(n, nnz, row_ptr, col_idx, true);
  if (prc != BCS_OK) return prc;
  std::vector<int> rp(row_ptr, row_ptr + n + 1), ci(col_idx, col_idx + nnz);
  IluProgram prog;
  if (!build_ilu_program(n, rp, ci, lanes, &prog))
    return fail(BCS_ERR_UNSUPPORTED, "positions of a pattern with %d entries do not fit 16 bits", nnz);
  if (nsteps) *nsteps = (int32_t)prog.widths.size();
  if (nwords) *nwords = (int32_t)prog.words.size();
  if (widths)
    for (size_t q = 0; q < prog.widths.size(); ++q) widths[q] = prog.widths[q];
  if (words)
    for (size_t q = 0; q < prog.words.size(); ++q) words[q] = prog.words[q];
  return BCS_OK;
}

static int check_common(const bcs_plan* p, int64_t ncells, const double* values, const double* gamma,
                        int64_t gamma_stride, double rtol, int32_t maxit) {
  if (!p) return fail(BCS_ERR_ARG, "plan is NULL");
  if (ncells < 0) return fail(BCS_ERR_ARG, "ncells must be >= 0");
  if (ncells > ((int64_t)1 << 40)) return fail(BCS_ERR_ARG, "ncells too large");
  if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(BCS_ERR_ARG, "rtol must be positive and finite");
  if (maxit < 1 || maxit > 1000000) return fail(BCS_ERR_ARG, "maxit must be in [1, 1000000]");
  if (ncells > 0 && !values) return fail(BCS_ERR_ARG, "values is NULL");
  if (p->opt.matrix_kind == BCS_J_GAMMA) {
    if (ncells > 0 && !gamma) return fail(BCS_ERR_ARG, "gamma is NULL");
    if (gamma_stride < 0) return fail(BCS_ERR_ARG, "gamma_stride must be >= 0");
  }
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess || cur != p->device)
    return fail(BCS_ERR_ARG, "the plan belongs to device %d, current device is %d", p->device, cur);
  return BCS_OK;
}

size_t bcs_workspace_bytes(const bcs_plan* p, int64_t ncells) {
  if (!p || ncells < 0) return 0;
  return ws_bytes(ncells);
}

int bcs_solve_batch(const bcs_plan* p, int64_t ncells, const double* values, const double* gamma,
                    int64_t gamma_stride, const double* b, const double* x0, double rtol, int32_t maxit, double* x,
                    int32_t* iters, double* resid, int32_t* status, int32_t* refinements, void* workspace,
                    size_t workspace_bytes, void* stream) {
  g_err.clear();
  int rc = check_common(p, ncells, values, gamma, gamma_stride, rtol, maxit);
  if (rc != BCS_OK) return rc;
  if (ncells == 0) return BCS_OK;
  if (!b || !x || !iters || !resid || !status) return fail(BCS_ERR_ARG, "b/x/iters/resid/status is NULL");
  if (x0 && p->opt.shared_scalars == 1)
    return fail(BCS_ERR_UNSUPPORTED, "shared_scalars plans take no initial guess");
  rc = check_workspace(p, ncells, workspace, workspace_bytes);
  if (rc != BCS_OK) return rc;
  bcs::KParams P = base_params(p, ncells, values, gamma, gamma_stride, rtol, maxit);
  P.b = b;
  P.x0 = x0;
  P.x = x;
  P.iters = iters;
  P.resid = resid;
  P.status = status;
  P.refinements = refinements;
  rc = prologue(p, &P, workspace, (hipStream_t)stream, slots_for(p, p->fwd, ncells), first_claims(p, p->fwd));
  if (rc != BCS_OK) return rc;
  return launch(p, p->fwd, P, (hipStream_t)stream);
}

int bcs_solve_batch_noalloc(const bcs_plan* p, int64_t ncells, const double* values, const double* gamma,
                            int64_t gamma_stride, const double* b, const double* x0, double rtol, int32_t maxit,
                            double* x, int32_t* iters, double* resid, int32_t* status, int32_t* refinements,
                            void* stream) {
  g_err.clear();
  int rc = check_common(p, ncells, values, gamma, gamma_stride, rtol, maxit);
  if (rc != BCS_OK) return rc;
  if (ncells == 0) return BCS_OK;
  if (ws_bytes(ncells) > (size_t)BCS_NOALLOC_MAX_BYTES)
    return fail(BCS_ERR_UNSUPPORTED, "%lld cells need %zu bytes of scratch, more than the %zu bytes of the "
                "no-allocation entry point (at most %lld cells)", (long long)ncells, ws_bytes(ncells),
                (size_t)BCS_NOALLOC_MAX_BYTES,
                (long long)(((size_t)BCS_NOALLOC_MAX_BYTES - bcs::kWsOrderOffset) / sizeof(int32_t)));
  void* ws = scratch_address(p->device);
  if (!ws) return fail(BCS_ERR_HIP, "no scratch address for device %d", p->device);
  return bcs_solve_batch(p, ncells, values, gamma, gamma_stride, b, x0, rtol, maxit, x, iters, resid, status,
                         refinements, ws, (size_t)BCS_NOALLOC_MAX_BYTES, stream);
}

int bcs_solve_batch_adjoint(const bcs_plan* p, int64_t ncells, const double* values, const double* gamma,
                            int64_t gamma_stride, const double* x, const double* g, double rtol, int32_t maxit,
                            int32_t grad_kind, double* grad_b, double* grad_vals, double* grad_gamma,
                            int32_t* iters, double* resid, int32_t* status, void* workspace,
                            size_t workspace_bytes, void* stream) {
  g_err.clear();
  int rc = check_common(p, ncells, values, gamma, gamma_stride, rtol, maxit);
  if (rc != BCS_OK) return rc;
  if (p->opt.shared_scalars == 1)
    return fail(BCS_ERR_UNSUPPORTED, "the adjoint is not available for shared_scalars plans");
  if (p->opt.precond == BCS_PRECOND_ILU0)
    return fail(BCS_ERR_UNSUPPORTED, "the adjoint is not available for ILU(0) plans");
  if (grad_kind != BCS_GRAD_A && grad_kind != BCS_GRAD_VALUES)
    return fail(BCS_ERR_ARG, "grad_kind must be BCS_GRAD_A or BCS_GRAD_VALUES");
  if (grad_gamma && p->opt.matrix_kind != BCS_J_GAMMA)
    return fail(BCS_ERR_ARG, "grad_gamma needs a BCS_J_GAMMA plan");
  if (ncells == 0) return BCS_OK;
  if (!x || !g || !grad_b || !grad_vals || !iters || !resid || !status)
    return fail(BCS_ERR_ARG, "x/g/grad_b/grad_vals/iters/resid/status is NULL");
  rc = check_workspace(p, ncells, workspace, workspace_bytes);
  if (rc != BCS_OK) return rc;
  bcs::KParams P = base_params(p, ncells, values, gamma, gamma_stride, rtol, maxit);
  P.b = g;
  P.x0 = nullptr;
  P.xin = x;
  P.x = grad_b;
  P.grad_kind = grad_kind == BCS_GRAD_VALUES ? 1 : 0;
  P.grad_vals = grad_vals;
  P.grad_gamma = grad_gamma;
  P.iters = iters;
  P.resid = resid;
  P.status = status;
  P.refinements = nullptr;
  rc = prologue(p, &P, workspace, (hipStream_t)stream, slots_for(p, p->adj, ncells), first_claims(p, p->adj));
  if (rc != BCS_OK) return rc;
  return launch(p, p->adj, P, (hipStream_t)stream);
}

size_t bcs_multi_workspace_bytes(int32_t nmech, const bcs_plan* const* plans, const int64_t* ncells) {
  if (nmech < 1 || nmech > bcs::kMaxMech || !plans || !ncells) return 0;
  size_t total = 0;
  for (int m = 0; m < nmech; ++m) {
    if (!plans[m] || ncells[m] < 0) return 0;
    total += ws_bytes(ncells[m]);
  }
  return total;
}

int bcs_solve_multi(int32_t nmech, const bcs_plan* const* plans, const int64_t* ncells,
                    const double* const* values, const double* const* gamma, const int64_t* gamma_stride,
                    const double* const* b, double rtol, int32_t maxit, double* const* x, int32_t* const* iters,
                    double* const* resid, int32_t* const* status, void* workspace, size_t workspace_bytes,
                    void* stream) {
  g_err.clear();
  if (nmech < 1 || nmech > bcs::kMaxMech) return fail(BCS_ERR_ARG, "nmech must be in [1, %d]", bcs::kMaxMech);
  if (!plans || !ncells || !values || !gamma || !gamma_stride || !b || !x || !iters || !resid || !status)
    return fail(BCS_ERR_ARG, "an array argument is NULL");
  std::vector<int> order;
  std::vector<size_t> ws_off(nmech, 0);  // each mechanism's part of the workspace, in argument order
  size_t ws_need = 0;
  for (int m = 0; m < nmech; ++m) {
    const bcs_plan* p = plans[m];
    int rc = check_common(p, ncells[m], values[m], gamma[m], gamma_stride[m], rtol, maxit);
    if (rc != BCS_OK) return rc;
    for (int q = 0; q < m; ++q)
      if (plans[q] == p) return fail(BCS_ERR_ARG, "a plan appears twice (mechanisms %d and %d)", q, m);
    if (p->opt.precision != BCS_FP64 || p->opt.jit != 1 || p->fwd.var || p->opt.shared_scalars == 1 ||
        p->opt.precond == BCS_PRECOND_ILU0)
      return fail(BCS_ERR_UNSUPPORTED,
                  "bcs_solve_multi needs FP64 plans created with jit = 1, shared_scalars = 0 and a Jacobi or no "
                  "preconditioner (mechanism %d)",
                  m);
    ws_off[m] = ws_need;
    ws_need += ws_bytes(ncells[m]);
    if (ncells[m] == 0) continue;
    if (!b[m] || !x[m] || !iters[m] || !resid[m] || !status[m])
      return fail(BCS_ERR_ARG, "b/x/iters/resid/status of mechanism %d is NULL", m);
    order.push_back(m);
  }
  if (order.empty()) return BCS_OK;
  if (!workspace) return fail(BCS_ERR_ARG, "workspace is NULL");
  if (((uintptr_t)workspace & 255u) != 0) return fail(BCS_ERR_ARG, "workspace must be 256-byte aligned");
  if (workspace_bytes < ws_need)
    return fail(BCS_ERR_ARG, "workspace of %zu bytes is smaller than the %zu bytes needed", workspace_bytes, ws_need);
  // heaviest cells first: their slots take longest, the light cells fill the tail
  std::stable_sort(order.begin(), order.end(), [&](int u, int v) {
    return (int64_t)plans[u]->fwd.ksteps * plans[u]->fwd.lanes > (int64_t)plans[v]->fwd.ksteps * plans[v]->fwd.lanes;
  });
  const int nm = (int)order.size();
  bcs::MultiParams M{};
  M.nmech = nm;
  // The mechanisms run one after another in each workgroup, so their slot
  // blocks share the operand and state regions (each sized for the largest
  // mechanism); every mechanism keeps its own tables.
  std::vector<WgLayout> lay(nm);
  int wxs = 0, wbs = 0;
  for (int q = 0; q < nm; ++q) {
    const Kernel& K = plans[order[q]]->fwd;
    lay[q] = wg_layout(plans[order[q]]->n, K.lanes, K.rpl, K.ksteps, 0);
    wxs = std::max(wxs, lay[q].wxs);
    wbs = std::max(wbs, lay[q].wbs);
  }
  const int operand = bcs::kWavesPerWg * wxs;
  size_t off = (size_t)operand + (size_t)bcs::kWavesPerWg * wbs;  // doubles
  for (int q = 0; q < nm; ++q) {
    const Kernel& K = plans[order[q]]->fwd;
    lay[q].wxs = wxs;
    lay[q].wbs = wbs;
    lay[q].bbase = operand;
    M.ent_off[q] = (int32_t)off;
    off += table_doubles(plans[order[q]]->n, K.lanes, K.ksteps);
  }
  // The gathers' 16-bit LDS addresses reach only the first 64 KiB: the
  // operand blocks must end below it, and the whole layout must fit the
  // device's LDS per workgroup.  Checked before anything is compiled.
  const size_t lds = off * 8;
  if ((size_t)operand * 8 > 65536 || lds > device_max_lds())
    return fail(BCS_ERR_UNSUPPORTED,
                "the mechanisms need %zu bytes of LDS per workgroup (%zu of them gathered operands), above the "
                "limit of %zu (operands: 65536)",
                lds, (size_t)operand * 8, device_max_lds());
  std::vector<int> lanes(nm), rpl(nm), flags(nm);
  std::vector<const int*> segs(nm);
  for (int q = 0; q < nm; ++q) {
    const Kernel& K = plans[order[q]]->fwd;
    lanes[q] = K.lanes;
    rpl[q] = K.rpl;
    flags[q] = K.flags;
    segs[q] = K.seg.data();
  }
  bcs::JitKernel jk;
  char err[512] = {0};
  int rc = bcs::jit_multi_kernel(nm, lanes.data(), flags.data(), segs.data(), rpl.data(), lds, &jk, err,
                                 sizeof(err));
  if (rc != BCS_OK) return fail(rc, "%s", err);
  int64_t need = 0;
  for (int q = 0; q < nm; ++q) {
    const int64_t cpw = (int64_t)bcs::kWavesPerWg * (64 / plans[order[q]]->fwd.lanes);
    need += (ncells[order[q]] + cpw - 1) / cpw;
  }
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)jk.max_blocks * plans[order[0]]->num_cu));
  for (int q = 0; q < nm; ++q) {
    const int m = order[q];
    const bcs_plan* p = plans[m];
    bcs::KParams P = base_params(p, ncells[m], values[m], gamma[m], gamma_stride[m], rtol, maxit);
    P.visits = nullptr;  // cell indices repeat across mechanisms
    P.b = b[m];
    P.x = x[m];
    P.iters = iters[m];
    P.resid = resid[m];
    P.status = status[m];
    P.refinements = nullptr;
    P.sched = p->fwd.d;
    P.adjoint = 0;
    P.xs = lay[q].xs;
    P.wxs = lay[q].wxs;
    P.bbase = lay[q].bbase;
    P.bs = lay[q].bs;
    P.wbs = lay[q].wbs;
    P.yoff = lay[q].yoff;
    P.tbase = M.ent_off[q];
    P.x0 = nullptr;
    // Every wave starts on the first mechanism: its cells are handed out
    // like a single mechanism's (slot k's first claim without the counter,
    // or slot k solves cell k when the grid has a slot for each); the
    // waves reach the others at different times and claim from their
    // counters, in each mechanism's own cost order.
    const int64_t slots = q == 0 ? (int64_t)grid * bcs::kWavesPerWg * (64 / p->fwd.lanes) : 0;
    rc = prologue(p, &P, (char*)workspace + ws_off[m], (hipStream_t)stream, slots, q == 0);
    if (rc != BCS_OK) return rc;
    M.m[q] = P;
  }
  void* args[] = {&M};
  const hipError_t e = hipModuleLaunchKernel(jk.fn, grid, 1, 1, bcs::kWgThreads, 1, 1, (unsigned)lds,
                                             (hipStream_t)stream, args, nullptr);
  if (e != hipSuccess) return fail(BCS_ERR_HIP, "multi launch: %s", hipGetErrorString(e));
  return BCS_OK;
}


int bcs_multi_autotune(int32_t nmech, bcs_plan* const* plans, const int64_t* ncells, const double* const* values,
                       const double* const* gamma, const int64_t* gamma_stride, const double* const* b,
                       double rtol, int32_t maxit, double* const* x, int32_t* const* iters, double* const* resid,
                       int32_t* const* status, int32_t* lanes_out) {
  g_err.clear();
  if (nmech < 1 || nmech > bcs::kMaxMech || !plans) return fail(BCS_ERR_ARG, "nmech must be in [1, %d]", bcs::kMaxMech);
  for (int m = 0; m < nmech; ++m)
    if (!plans[m]) return fail(BCS_ERR_ARG, "plan %d is NULL", m);
  if (hipDeviceSynchronize() != hipSuccess) return fail(BCS_ERR_HIP, "device synchronisation failed");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(BCS_ERR_HIP, "multi autotune: event creation failed");
  }
  const bcs_plan* const* cplans = plans;
  OwnedWorkspace ws;
  const size_t ws_need = bcs_multi_workspace_bytes(nmech, cplans, ncells);
  if (ws_need == 0) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return fail(BCS_ERR_ARG, "bad cell counts");
  }
  if (ws.alloc(ws_need) != BCS_OK) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return BCS_ERR_HIP;
  }
  // one combined launch as the plans stand: a warm-up (which also compiles the
  // combination), then the best of two timed launches
  auto time_multi = [&](double* secs) -> int {
    int rc = bcs_solve_multi(nmech, cplans, ncells, values, gamma, gamma_stride, b, rtol, maxit, x, iters, resid,
                             status, ws.ptr, ws_need, nullptr);
    if (rc != BCS_OK) return rc;
    double best = 1e300;
    for (int rep = 0; rep < 2; ++rep) {
      (void)hipEventRecord(e0, nullptr);
      rc = bcs_solve_multi(nmech, cplans, ncells, values, gamma, gamma_stride, b, rtol, maxit, x, iters, resid,
                           status, ws.ptr, ws_need, nullptr);
      if (rc != BCS_OK) return rc;
      (void)hipEventRecord(e1, nullptr);
      if (hipEventSynchronize(e1) != hipSuccess) return fail(BCS_ERR_HIP, "multi autotune: synchronisation failed");
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      best = std::min(best, (double)ms * 1e-3);
    }
    *secs = best;
    return BCS_OK;
  };
  double best = 0;
  int rc = time_multi(&best);
  // coordinate descent: each mechanism in turn tries the other lane counts
  // with the others held, keeping any that shortens the combined launch
  for (int pass = 0; rc == BCS_OK && pass < 2; ++pass) {
    bool improved = false;
    for (int m = 0; rc == BCS_OK && m < nmech; ++m) {
      bcs_plan* p = plans[m];
      if (p->opt.lanes_per_cell != 0 || ncells[m] == 0) continue;  // fixed by the caller, or nothing to time
      std::vector<int> pos(p->nnz), trp, tci, tpos;
      for (int k = 0; k < p->nnz; ++k) pos[k] = k;
      transpose_pattern(p->n, p->rp, p->ci, trp, tci, tpos);
      for (int L : {16, 32, 64}) {
        if (L == p->fwd.lanes || !adjoint_fits(p->n, trp, tci, tpos, L)) continue;
        Kernel K;
        g_err.clear();
        int r = make_kernel(p->n, p->rp, p->ci, pos, L, 0, p->opt.jit == 1, 0, false, &K);
        if (r == BCS_ERR_UNSUPPORTED && g_err.empty()) continue;
        if (r != BCS_OK) {
          rc = r;
          break;
        }
        Kernel keep = p->fwd;
        p->fwd = K;
        double t = 0;
        r = time_multi(&t);
        if (verbose()) std::fprintf(stderr, "[bcs] multi autotune mechanism %d lanes=%d: %.1f us\n", m, L, t * 1e6);
        if (r == BCS_OK && t < best) {
          best = t;
          free_kernel(&keep);
          improved = true;
        } else {
          p->fwd = keep;
          free_kernel(&K);
          if (r != BCS_OK) {
            rc = r;
            break;
          }
        }
      }
    }
    if (!improved) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != BCS_OK) return rc;
  // the adjoint kernels follow the chosen lane counts
  for (int m = 0; m < nmech; ++m) {
    bcs_plan* p = plans[m];
    if (p->adj.lanes != p->fwd.lanes) {
      std::vector<int> trp, tci, tpos;
      transpose_pattern(p->n, p->rp, p->ci, trp, tci, tpos);
      Kernel A;
      g_err.clear();
      rc = make_kernel(p->n, trp, tci, tpos, p->fwd.lanes, 1, p->opt.jit == 1, 0, false, &A);
      if (rc != BCS_OK) return g_err.empty() ? fail(rc, "no kernel layout holds the transposed pattern") : rc;
      free_kernel(&p->adj);
      p->adj = A;
    }
    const int r = sync_mech(p);
    if (r != BCS_OK) return r;
    if (lanes_out) lanes_out[m] = p->fwd.lanes;
  }
  return BCS_OK;
}

void bcs_debug_count_visits(int32_t* counts) { g_visits = counts; }

int bcs_plan_create_mech(const bcs_mechanism* mech, const bcs_options* opt, bcs_plan** out) {
  g_err.clear();
  if (!out) return fail(BCS_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!mech) return fail(BCS_ERR_ARG, "mechanism is NULL");
  bcs_options o;
  bcs_options_default(&o);
  if (opt) o = *opt;
  if (o.precision != BCS_FP64 || (o.precond != BCS_PRECOND_NONE && o.precond != BCS_PRECOND_JACOBI) ||
      o.matrix_kind != BCS_J_GAMMA || o.jit != 1 || o.shared_scalars != 0)
    return fail(BCS_ERR_UNSUPPORTED, "a mechanism plan needs FP64, no or Jacobi preconditioning, J_GAMMA, jit = 1 "
                "and shared_scalars = 0");
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess || cur != mech->device)
    return fail(BCS_ERR_ARG, "the mechanism belongs to device %d", mech->device);
  bcs_plan* p = nullptr;
  int rc = bcs_plan_create(mech->n, mech->nnz, mech->rp.data(), mech->ci.data(), &o, &p);
  if (rc != BCS_OK) return rc;
  p->mech = mech;
  rc = sync_mech(p);
  if (rc != BCS_OK) {
    release(p);
    return rc;
  }
  *out = p;
  return BCS_OK;
}

int bcs_solve_batch_mech(const bcs_plan* p, int64_t ncells, const double* y, const double* k, int64_t k_stride,
                         const double* gamma, int64_t gamma_stride, const double* b, const double* x0, double rtol,
                         int32_t maxit, double* x, int32_t* iters, double* resid, int32_t* status, void* workspace,
                         size_t workspace_bytes, void* stream) {
  g_err.clear();
  int rc = check_common(p, ncells, y, gamma, gamma_stride, rtol, maxit);
  if (rc != BCS_OK) return rc;
  if (!p->mech || !p->fwd_mech.buf) return fail(BCS_ERR_UNSUPPORTED, "the plan was not made from a mechanism");
  if (k_stride != 0 && k_stride < p->mech->R) return fail(BCS_ERR_ARG, "k_stride must be 0 or at least nreact");
  if (ncells == 0) return BCS_OK;
  if (!k || !b || !x || !iters || !resid || !status) return fail(BCS_ERR_ARG, "k/b/x/iters/resid/status is NULL");
  rc = check_workspace(p, ncells, workspace, workspace_bytes);
  if (rc != BCS_OK) return rc;
  bcs::KParams P = base_params(p, ncells, y, gamma, gamma_stride, rtol, maxit);
  P.b = b;
  P.x0 = x0;
  P.x = x;
  P.iters = iters;
  P.resid = resid;
  P.status = status;
  P.refinements = nullptr;
  P.y = y;
  P.kr = k;
  P.k_stride = k_stride;
  P.mtab = (const int32_t*)p->fwd_mech.mbuf;
  P.mtab_words = p->fwd_mech.mwords;
  P.mk = k_stride == 0 ? p->mech->R : 0;
  P.mr = p->mech->R;
  rc = prologue(p, &P, workspace, (hipStream_t)stream, slots_for(p, p->fwd_mech, ncells), first_claims(p, p->fwd_mech));
  if (rc != BCS_OK) return rc;
  return launch(p, p->fwd_mech, P, (hipStream_t)stream);
}

}  // extern "C"
