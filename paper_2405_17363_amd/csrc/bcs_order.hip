// Cost order of the cells of a J_GAMMA solve: a two-pass counting sort of the
// cell indices by a bucket of gamma, largest gamma first.  A cell's
// iteration count grows with gamma (A = I - gamma J drifts away from the
// identity), so handing the cells out in this order lets the expensive cells
// start early.  Within a bucket the order is whatever the atomics give; a
// cell's results do not depend on when or where it is solved.
#include "bcs_internal.h"

namespace bcs {
namespace {

constexpr int kOrderThreads = 256;
constexpr int kCellsPerThread = 4;
constexpr int kCellsPerBlock = kOrderThreads * kCellsPerThread;

// Bucket of a gamma value: the IEEE-754 bits of a positive double, shifted
// to keep the exponent and the two leading mantissa bits, are monotone in
// the value (a quarter octave per step).  Bucket 0 holds gamma <= 2^-16, zero,
// negative and NaN values; the last bucket everything from 2^16 up.
__device__ __forceinline__ int gamma_bucket(double g) {
  if (!(g > 0.0)) return 0;
  const long long q = (long long)(__builtin_bit_cast(unsigned long long, g) >> 50);
  const long long q0 = (long long)(1023 - 16) << 2;
  const long long b = q - q0;
  return b < 0 ? 0 : (b >= kOrderBuckets ? kOrderBuckets - 1 : (int)b);
}

// Pass 0: clear the solve's work queue (the claim counter starts at qstart,
// the positions the slots' first claims take without it) and, when a cost
// order is built, the sort state.  A kernel, not a memset, so that the whole prologue is plain
// kernel launches on the solve's stream.
__global__ void __launch_bounds__(kOrderThreads) k_order_clear(unsigned long long* queue, unsigned long long qstart,
                                                               uint32_t* state) {
  for (int i = threadIdx.x; i < kQueueWords; i += kOrderThreads) queue[i] = i == 0 ? qstart : 0ull;
  if (state)
    for (int i = threadIdx.x; i < kOrderStateWords; i += kOrderThreads) state[i] = 0u;
}

// Pass 1: count the cells of every bucket (state[0 .. kOrderBuckets)).
__global__ void __launch_bounds__(kOrderThreads) k_order_count(const double* gamma, int64_t stride, int64_t ncells,
                                                               uint32_t* state) {
  __shared__ uint32_t cnt[kOrderBuckets];
  for (int i = threadIdx.x; i < kOrderBuckets; i += kOrderThreads) cnt[i] = 0u;
  __syncthreads();
  const int64_t c0 = (int64_t)blockIdx.x * kCellsPerBlock;
  for (int q = 0; q < kCellsPerThread; ++q) {
    const int64_t c = c0 + (int64_t)q * kOrderThreads + threadIdx.x;
    if (c < ncells) atomicAdd(&cnt[gamma_bucket(gamma[c * stride])], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kOrderBuckets; i += kOrderThreads)
    if (cnt[i]) atomicAdd(&state[i], cnt[i]);
}

// Pass 2: the start of every bucket in the output (buckets in decreasing
// order, i.e. decreasing gamma), a range per block and bucket claimed from
// the bucket cursors (state[kOrderBuckets ..)), then every cell written to
// its place.
__global__ void __launch_bounds__(kOrderThreads) k_order_scatter(const double* gamma, int64_t stride, int64_t ncells,
                                                                 uint32_t* state, int32_t* order) {
  __shared__ uint32_t start[kOrderBuckets];
  __shared__ uint32_t cnt[kOrderBuckets];
  __shared__ uint32_t base[kOrderBuckets];
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (int b = kOrderBuckets - 1; b >= 0; --b) {
      start[b] = s;
      s += state[b];
    }
  }
  for (int i = threadIdx.x; i < kOrderBuckets; i += kOrderThreads) cnt[i] = 0u;
  __syncthreads();
  const int64_t c0 = (int64_t)blockIdx.x * kCellsPerBlock;
  int bucket[kCellsPerThread];
  uint32_t local[kCellsPerThread];
  for (int q = 0; q < kCellsPerThread; ++q) {
    const int64_t c = c0 + (int64_t)q * kOrderThreads + threadIdx.x;
    bucket[q] = -1;
    if (c < ncells) {
      bucket[q] = gamma_bucket(gamma[c * stride]);
      local[q] = atomicAdd(&cnt[bucket[q]], 1u);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kOrderBuckets; i += kOrderThreads)
    base[i] = cnt[i] ? start[i] + atomicAdd(&state[kOrderBuckets + i], cnt[i]) : 0u;
  __syncthreads();
  for (int q = 0; q < kCellsPerThread; ++q) {
    const int64_t c = c0 + (int64_t)q * kOrderThreads + threadIdx.x;
    if (bucket[q] >= 0) order[base[bucket[q]] + local[q]] = (int32_t)c;
  }
}

}  // namespace

hipError_t launch_solve_prologue(unsigned long long* queue, unsigned long long qstart, const double* gamma,
                                 int64_t stride, int64_t ncells, uint32_t* state, int32_t* order, hipStream_t stream) {
  hipLaunchKernelGGL(k_order_clear, dim3(1), dim3(kOrderThreads), 0, stream, queue, qstart, order ? state : nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !order) return e;
  const int blocks = (int)((ncells + kCellsPerBlock - 1) / kCellsPerBlock);
  hipLaunchKernelGGL(k_order_count, dim3(blocks), dim3(kOrderThreads), 0, stream, gamma, stride, ncells, state);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_order_scatter, dim3(blocks), dim3(kOrderThreads), 0, stream, gamma, stride, ncells, state,
                     order);
  return hipGetLastError();
}

}  // namespace bcs
