// Mass-action rates and Jacobian of every cell, on the device: the inputs of
// the batched linear solve (Section 2.1: the rate of change of each species
// is a sum of reaction contributions per cell, and the BDF integrator needs
// the Jacobian of that rate function on its shared sparse pattern; Section 6
// names moving the rest of the BDF step onto the GPU as the next step).
//
// A mechanism is a list of reactions with one or two reactants and up to two
// products.  Reaction r runs at w_r = k_r y_a (one reactant) or
// (k_r y_a) y_b (two, a == b allowed); species i changes at
// f_i = sum_r S_ir w_r (S_ir = products minus reactants) and
// J_ij = sum_r S_ir dw_r/dy_j, with dw/dy_a = k_r (one reactant),
// k_r y_b and k_r y_a (a != b), 2 (k_r y_a) (a == b).
//
// The host turns the mechanism into gather lists once: for every CSR
// position of the pattern, the reactions that contribute to it (reaction,
// S_ir, the other reactant or none, the factor 2), in increasing reaction
// order; for every species, the reactions that change it (reaction, S_ir).
// A workgroup then takes up to eight consecutive cells at a time (fewer when
// the staging would not fit the LDS), stages their
// concentrations (and per-cell rate constants) in LDS with coalesced loads;
// a thread then takes a position (a species, for f) and, reading its term
// list once, accumulates it for all the staged cells, so consecutive threads
// write consecutive addresses of every cell's row.  Every sum runs over its terms in increasing reaction order,
// each term's product S_ir * (k_r ...) exact (S_ir is a small integer), so
// the results are bitwise those of summing reaction by reaction.
#include <algorithm>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "bcs_internal.h"

namespace bcs {
namespace {

constexpr int kAsmThreads = 256;
constexpr int kAsmCellsMax = 8;    // most cells a workgroup stages at a time

// J term: word 0 = reaction; word 1 = other reactant (16 bits, kNoSpecies =
// none) | (S_ir + 128) << 16 | factor-2 flag << 24.
// f term: word 0 = reaction; word 1 = S_ir + 128.
struct AsmParams {
  int64_t ncells;
  int n, nnz, R;
  int cells;  // cells staged at a time
  const double* y;
  const double* k;
  int64_t k_stride;
  double* f;
  double* J;
  const int32_t* tables;  // the mechanism's tables, copied into LDS
  int table_words;
  int jofs, jterm, fofs, fterm, reac;  // word offsets of the tables
};

__global__ void __launch_bounds__(kAsmThreads) k_assemble(AsmParams P) {
  extern __shared__ double lds[];
  const int n = P.n, nnz = P.nnz, R = P.R;
  const bool kcell = P.k_stride != 0;
  const int CB = P.cells;
  // LDS: y [CB][n], k [CB or 1][R], w [CB][R] (rates, for f), tables
  double* ys = lds;
  double* ks = ys + CB * n;
  double* ws = ks + (kcell ? CB : 1) * R;
  int32_t* tab = (int32_t*)(ws + (P.f ? CB * R : 0));
  for (int i = threadIdx.x; i < P.table_words; i += kAsmThreads) tab[i] = P.tables[i];
  if (!kcell)
    for (int r = threadIdx.x; r < R; r += kAsmThreads) ks[r] = P.k[r];
  const int32_t* jofs = tab + P.jofs;
  const int32_t* jterm = tab + P.jterm;
  const int32_t* fofs = tab + P.fofs;
  const int32_t* fterm = tab + P.fterm;
  const int32_t* reac = tab + P.reac;

  const int64_t nblk = (P.ncells + CB - 1) / CB;
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t c0 = blk * CB;
    const int nc = (int)((P.ncells - c0) < CB ? (P.ncells - c0) : CB);
    __syncthreads();  // the previous block's readers are done (and the tables are in)
    // the cells' concentrations are contiguous: nc * n doubles
    for (int i = threadIdx.x; i < nc * n; i += kAsmThreads) ys[i] = P.y[c0 * n + i];
    if (kcell)
      for (int i = threadIdx.x; i < nc * R; i += kAsmThreads) {
        const int cc = i / R, r = i - cc * R;
        ks[i] = P.k[(c0 + cc) * P.k_stride + r];
      }
    __syncthreads();
    if (P.f) {
      // reaction rates w_r = k_r y_a (y_b)
      for (int i = threadIdx.x; i < nc * R; i += kAsmThreads) {
        const int cc = i / R, r = i - cc * R;
        const double* yc = ys + cc * n;
        const double kr = ks[(kcell ? cc * R : 0) + r];
        const int a = reac[2 * r], b = reac[2 * r + 1];
        double w = kr * yc[a];
        if (b >= 0) w = w * yc[b];
        ws[i] = w;
      }
      __syncthreads();
      // species i of every staged cell: one pass over i's terms
      for (int i = threadIdx.x; i < n; i += kAsmThreads) {
        double acc[kAsmCellsMax];
#pragma unroll
        for (int cc = 0; cc < kAsmCellsMax; ++cc) acc[cc] = 0.0;
        for (int t = fofs[i]; t < fofs[i + 1]; ++t) {
          const int r = fterm[2 * t];
          const double s = (double)(fterm[2 * t + 1] - 128);
#pragma unroll
          for (int cc = 0; cc < kAsmCellsMax; ++cc)
            if (cc < nc) acc[cc] = __builtin_fma(s, ws[cc * R + r], acc[cc]);  // s * w is exact
        }
#pragma unroll
        for (int cc = 0; cc < kAsmCellsMax; ++cc)
          if (cc < nc) P.f[(c0 + cc) * n + i] = acc[cc];
      }
    }
    if (P.J) {
      // position q of every staged cell: one pass over q's terms, the term
      // words read once for all the cells; consecutive threads write
      // consecutive positions of each cell's row
      for (int q = threadIdx.x; q < nnz; q += kAsmThreads) {
        double acc[kAsmCellsMax];
#pragma unroll
        for (int cc = 0; cc < kAsmCellsMax; ++cc) acc[cc] = 0.0;
        for (int t = jofs[q]; t < jofs[q + 1]; ++t) {
          const int r = jterm[2 * t];
          const uint32_t w1 = (uint32_t)jterm[2 * t + 1];
          const int other = (int)(w1 & 0xffffu);
          const double s = (double)((int)((w1 >> 16) & 0xffu) - 128);
          const bool dbl = (w1 >> 24) != 0;
          const double ksh = ks[r];  // the shared rate constant (unused with per-cell ones)
#pragma unroll
          for (int cc = 0; cc < kAsmCellsMax; ++cc)
            if (cc < nc) {
              double d = kcell ? ks[cc * R + r] : ksh;
              if (other != kNoSpecies) d = d * ys[cc * n + other];
              if (dbl) d = d * 2.0;                     // 2 (k y_a): exact doubling
              acc[cc] = __builtin_fma(s, d, acc[cc]);   // s * d is exact
            }
        }
#pragma unroll
        for (int cc = 0; cc < kAsmCellsMax; ++cc)
          if (cc < nc) P.J[(c0 + cc) * nnz + q] = acc[cc];
      }
    }
  }
}

int asm_fail(int code, const std::string& msg) { return set_error(code, msg.c_str()); }

size_t lds_bytes(const bcs_mechanism* m, int cells, bool per_cell_k, bool with_f) {
  const size_t dbl = (size_t)cells * m->n + (size_t)(per_cell_k ? cells : 1) * m->R +
                     (with_f ? (size_t)cells * m->R : 0);
  return dbl * sizeof(double) + m->table_words * sizeof(int32_t);
}

}  // namespace

}  // namespace bcs

extern "C" {

int bcs_mechanism_create(int32_t n, int32_t nnz, const int32_t* row_ptr, const int32_t* col_idx, int32_t nreact,
                         const int32_t* reactants, const int32_t* products, bcs_mechanism** out) {
  using bcs::asm_fail;
  bcs::clear_error();
  if (!out) return asm_fail(BCS_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (n <= 0 || n >= bcs::kNoSpecies) return asm_fail(BCS_ERR_ARG, "n must be in [1, 65534]");
  if (nnz < 1 || nreact < 1 || nreact > (1 << 24)) return asm_fail(BCS_ERR_ARG, "nnz and nreact must be positive");
  if (!row_ptr || !col_idx || !reactants || !products)
    return asm_fail(BCS_ERR_ARG, "row_ptr/col_idx/reactants/products is NULL");
  if (row_ptr[0] != 0 || row_ptr[n] != nnz) return asm_fail(BCS_ERR_PATTERN, "row_ptr[0] must be 0 and row_ptr[n] nnz");
  for (int i = 0; i < n; ++i) {
    if (row_ptr[i + 1] < row_ptr[i]) return asm_fail(BCS_ERR_PATTERN, "row_ptr decreases");
    for (int q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
      if (col_idx[q] < 0 || col_idx[q] >= n) return asm_fail(BCS_ERR_PATTERN, "column index out of range");
      if (q > row_ptr[i] && col_idx[q] <= col_idx[q - 1])
        return asm_fail(BCS_ERR_PATTERN, "columns not strictly increasing within a row");
    }
  }
  auto pos_of = [&](int i, int j) {
    for (int q = row_ptr[i]; q < row_ptr[i + 1]; ++q)
      if (col_idx[q] == j) return q;
    return -1;
  };
  // per-position and per-species term lists, in reaction order
  std::vector<std::vector<std::pair<int, uint32_t>>> jt(nnz), ft(n);
  for (int r = 0; r < nreact; ++r) {
    const int a = reactants[2 * r], b = reactants[2 * r + 1];
    if (a < 0 || a >= n || b < -1 || b >= n)
      return asm_fail(BCS_ERR_ARG, "reaction " + std::to_string(r) + ": reactant out of range (first must be given)");
    const int all[4] = {a, b, products[2 * r], products[2 * r + 1]};
    if (all[2] < -1 || all[2] >= n || all[3] < -1 || all[3] >= n)
      return asm_fail(BCS_ERR_ARG, "reaction " + std::to_string(r) + ": product out of range");
    // species of the reaction (each once) with their net stoichiometry
    int sp[4], st[4], ns = 0;
    for (int q = 0; q < 4; ++q) {
      if (all[q] < 0) continue;
      const int d = q < 2 ? -1 : 1;
      int u = 0;
      while (u < ns && sp[u] != all[q]) ++u;
      if (u == ns) {
        sp[ns] = all[q];
        st[ns++] = d;
      } else {
        st[u] += d;
      }
    }
    // derivatives of w_r: (species j, other reactant or none, factor 2)
    int dj[2], other[2], dbl[2], nd;
    if (b < 0) {
      dj[0] = a, other[0] = bcs::kNoSpecies, dbl[0] = 0, nd = 1;
    } else if (a == b) {
      dj[0] = a, other[0] = a, dbl[0] = 1, nd = 1;
    } else {
      dj[0] = a, other[0] = b, dbl[0] = 0;
      dj[1] = b, other[1] = a, dbl[1] = 0, nd = 2;
    }
    for (int u = 0; u < ns; ++u) {
      ft[sp[u]].push_back({r, (uint32_t)(st[u] + 128)});
      for (int v = 0; v < nd; ++v) {
        const int q = pos_of(sp[u], dj[v]);
        if (q < 0)
          return asm_fail(BCS_ERR_PATTERN, "reaction " + std::to_string(r) + " needs pattern entry (" +
                                               std::to_string(sp[u]) + ", " + std::to_string(dj[v]) +
                                               "), which the pattern lacks");
        jt[q].push_back({r, (uint32_t)other[v] | ((uint32_t)(st[u] + 128) << 16) | ((uint32_t)dbl[v] << 24)});
      }
    }
  }
  std::vector<int32_t> tab;
  const int jofs = 0;
  tab.resize(nnz + 1);
  int nj = 0;
  for (int q = 0; q < nnz; ++q) {
    tab[jofs + q] = nj;
    nj += (int)jt[q].size();
  }
  tab[jofs + nnz] = nj;
  const int jterm = (int)tab.size();
  for (int q = 0; q < nnz; ++q)
    for (auto& t : jt[q]) {
      tab.push_back(t.first);
      tab.push_back((int32_t)t.second);
    }
  const int fofs = (int)tab.size();
  int nf = 0;
  for (int i = 0; i < n; ++i) {
    tab.push_back(nf);
    nf += (int)ft[i].size();
  }
  tab.push_back(nf);
  const int fterm = (int)tab.size();
  for (int i = 0; i < n; ++i)
    for (auto& t : ft[i]) {
      tab.push_back(t.first);
      tab.push_back((int32_t)t.second);
    }
  const int reac = (int)tab.size();
  for (int r = 0; r < 2 * nreact; ++r) tab.push_back(reactants[r]);

  bcs_mechanism* m = new bcs_mechanism();
  m->n = n, m->nnz = nnz, m->R = nreact, m->nj = nj, m->nf = nf;
  m->rp.assign(row_ptr, row_ptr + n + 1);
  m->ci.assign(col_idx, col_idx + nnz);
  m->table_words = tab.size();
  m->htab = tab;
  m->jofs_at = jofs;
  m->jterm_at = jterm;
  if (hipGetDevice(&m->device) != hipSuccess ||
      hipDeviceGetAttribute(&m->num_cu, hipDeviceAttributeMultiprocessorCount, m->device) != hipSuccess) {
    delete m;
    return asm_fail(BCS_ERR_HIP, "no HIP device");
  }
  hipError_t e = hipMalloc((void**)&m->buf, tab.size() * sizeof(int32_t));
  if (e == hipSuccess) e = hipMemcpy(m->buf, tab.data(), tab.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (m->buf) (void)hipFree(m->buf);
    delete m;
    return asm_fail(BCS_ERR_HIP, std::string("mechanism tables: ") + hipGetErrorString(e));
  }
  m->jofs = m->buf + jofs;
  m->jterm = m->buf + jterm;
  m->fofs = m->buf + fofs;
  m->fterm = m->buf + fterm;
  m->reac = m->buf + reac;
  *out = m;
  return BCS_OK;
}

void bcs_mechanism_destroy(bcs_mechanism* m) {
  if (!m) return;
  int cur = 0;
  if (hipGetDevice(&cur) == hipSuccess && cur != m->device) (void)hipSetDevice(m->device);
  if (m->buf) (void)hipFree(m->buf);
  if (cur != m->device) (void)hipSetDevice(cur);
  delete m;
}

int bcs_assemble(const bcs_mechanism* m, int64_t ncells, const double* y, const double* k, int64_t k_stride,
                 double* f, double* J, void* stream) {
  using bcs::asm_fail;
  bcs::clear_error();
  if (!m) return asm_fail(BCS_ERR_ARG, "mechanism is NULL");
  if (ncells < 0) return asm_fail(BCS_ERR_ARG, "ncells must be >= 0");
  if (k_stride != 0 && k_stride < m->R) return asm_fail(BCS_ERR_ARG, "k_stride must be 0 or at least nreact");
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess || cur != m->device)
    return asm_fail(BCS_ERR_ARG, "the mechanism belongs to another device");
  if (ncells == 0 || (!f && !J)) return BCS_OK;
  if (!y || !k) return asm_fail(BCS_ERR_ARG, "y/k is NULL");
  int cells = bcs::kAsmCellsMax;
  while (cells > 1 && bcs::lds_bytes(m, cells, k_stride != 0, f != nullptr) > 64 * 1024) cells /= 2;
  const size_t lds = bcs::lds_bytes(m, cells, k_stride != 0, f != nullptr);
  if (lds > 64 * 1024)
    return asm_fail(BCS_ERR_UNSUPPORTED, "the mechanism's tables and staging need " + std::to_string(lds) +
                                             " bytes of LDS per workgroup (limit 65536)");
  bcs::AsmParams P{};
  P.ncells = ncells;
  P.n = m->n, P.nnz = m->nnz, P.R = m->R;
  P.cells = cells;
  P.y = y, P.k = k, P.k_stride = k_stride, P.f = f, P.J = J;
  P.tables = m->buf;
  P.table_words = (int)m->table_words;
  P.jofs = (int)(m->jofs - m->buf), P.jterm = (int)(m->jterm - m->buf), P.fofs = (int)(m->fofs - m->buf);
  P.fterm = (int)(m->fterm - m->buf), P.reac = (int)(m->reac - m->buf);
  const int64_t nblk = (ncells + cells - 1) / cells;
  // enough resident workgroups to keep every CU's memory pipeline busy
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(nblk, (int64_t)m->num_cu * 8));
  hipLaunchKernelGGL(bcs::k_assemble, dim3(grid), dim3(bcs::kAsmThreads), lds, (hipStream_t)stream, P);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return asm_fail(BCS_ERR_HIP, std::string("assemble launch: ") + hipGetErrorString(e));
  return BCS_OK;
}

}  // extern "C"
