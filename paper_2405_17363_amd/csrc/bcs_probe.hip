// Measured ceilings of the resources the solve kernels use: HBM streaming,
// the LDS gather of FP64 operands, and the FP64 / FP32 vector FMA rate.  The
// roofline of the batched solve is set by whichever of these its work
// exhausts first, and the published peaks (or the ones derived from unit
// counts and clock) are what the hardware could do at best; these kernels
// measure what a plain, well-formed kernel attains.  The caller times the
// launches (HIP events on `stream`) and divides the bytes or flops each
// launch performs, returned by the functions below, by the time.
#include "bcs_device.h"
#include "bcs_internal.h"
#include "../../include/bcs_probe.h"

namespace bcs {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kLdsDoubles = 4096;  // 32 KiB of LDS per workgroup
constexpr int kProbeUnroll = 16;   // independent loads / FMA chains per thread

// out[i] = in[i], vectorised by 2 doubles per thread and grid-strided.
__global__ void __launch_bounds__(kProbeThreads) k_copy(const double2* __restrict__ in, double2* __restrict__ out,
                                                      int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
  for (int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x; i < n2; i += stride) out[i] = in[i];
}

// Every thread gathers kProbeUnroll FP64 words from the workgroup's LDS per
// round, `rounds` rounds.  pattern 0: the 64 lanes of a wave read 64
// consecutive words (no bank conflicts); pattern 1: each lane reads a
// pseudo-random word (a multiplicative hash of its round, slot and lane),
// like the solve's gathers of random columns.  All addresses stay inside
// the kLdsDoubles-word array.
template <int PATTERN>
__global__ void __launch_bounds__(kProbeThreads) k_lds(double* out, int64_t rounds) {
  __shared__ double buf[kLdsDoubles];
  for (int i = threadIdx.x; i < kLdsDoubles; i += kProbeThreads) buf[i] = (double)(i & 7);
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double acc[kProbeUnroll];
#pragma unroll
  for (int u = 0; u < kProbeUnroll; ++u) acc[u] = 0.0;
  for (int64_t r = 0; r < rounds; ++r) {
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) {
      // k runs over the array's 64 blocks of 64 words as r advances (an odd
      // step, so no load repeats the previous round's and none can be hoisted)
      const uint32_t k = (uint32_t)r * (kProbeUnroll * 4u + 1u) + u * 4u + wv;
      const uint32_t idx = PATTERN == 0 ? ((k & 63u) * 64u + lane) : ((k * 64u + lane) * 2654435761u) >> 20;
      acc[u] += buf[idx & (kLdsDoubles - 1)];
    }
  }
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < kProbeUnroll; ++u) s += acc[u];
  out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

// kProbeUnroll independent FMA chains per thread, `rounds` steps each.
template <typename T>
__global__ void __launch_bounds__(kProbeThreads) k_fma(T* out, int64_t rounds, T a, T b) {
  T v[kProbeUnroll];
#pragma unroll
  for (int u = 0; u < kProbeUnroll; ++u) v[u] = (T)(threadIdx.x + u);
  for (int64_t r = 0; r < rounds; ++r) {
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) v[u] = dev::fmat(v[u], a, b);
  }
  T s = 0;
#pragma unroll
  for (int u = 0; u < kProbeUnroll; ++u) s += v[u];
  out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

}  // namespace
}  // namespace bcs

extern "C" {

int bcs_probe_threads_per_block(void) { return bcs::kProbeThreads; }

double bcs_probe_copy(const double* in, double* out, int64_t n, int32_t blocks, void* stream) {
  if (!in || !out || n < 2 || (n & 1) || blocks < 1) return -1.0;
  hipLaunchKernelGGL(bcs::k_copy, dim3(blocks), dim3(bcs::kProbeThreads), 0, (hipStream_t)stream,
                     (const double2*)in, (double2*)out, n / 2);
  if (hipGetLastError() != hipSuccess) return -1.0;
  return 16.0 * (double)n;
}

double bcs_probe_lds(double* out, int64_t rounds, int32_t pattern, int32_t blocks, void* stream) {
  if (!out || rounds < 1 || blocks < 1 || (pattern != 0 && pattern != 1)) return -1.0;
  if (pattern == 0)
    hipLaunchKernelGGL(bcs::k_lds<0>, dim3(blocks), dim3(bcs::kProbeThreads), 0, (hipStream_t)stream, out, rounds);
  else
    hipLaunchKernelGGL(bcs::k_lds<1>, dim3(blocks), dim3(bcs::kProbeThreads), 0, (hipStream_t)stream, out, rounds);
  if (hipGetLastError() != hipSuccess) return -1.0;
  return 8.0 * bcs::kProbeUnroll * (double)rounds * bcs::kProbeThreads * blocks;
}

double bcs_probe_fma(void* out, int64_t rounds, int32_t fp64, int32_t blocks, void* stream) {
  if (!out || rounds < 1 || blocks < 1) return -1.0;
  if (fp64)
    hipLaunchKernelGGL(bcs::k_fma<double>, dim3(blocks), dim3(bcs::kProbeThreads), 0, (hipStream_t)stream,
                       (double*)out, rounds, 0.999999, 1e-7);
  else
    hipLaunchKernelGGL(bcs::k_fma<float>, dim3(blocks), dim3(bcs::kProbeThreads), 0, (hipStream_t)stream,
                       (float*)out, rounds, 0.999999f, 1e-7f);
  if (hipGetLastError() != hipSuccess) return -1.0;
  return 2.0 * bcs::kProbeUnroll * (double)rounds * bcs::kProbeThreads * blocks;
}

}  // extern "C"
