/* bcs_probe.h -- measured ceilings for the roofline of the batched solve.
 *
 * The solve's work per cell is compulsory HBM traffic (its values, right-hand
 * side and outputs), FP64 (or FP32) vector FMAs, and gathers of SpMV
 * operands from LDS (Section 3.1's solver keeps a cell in one block; here a
 * cell's operand vector lives in LDS and every stored matrix entry gathers
 * one word per SpMV).  These launches measure what a plain kernel attains
 * on each of those resources, to stand beside the published or derived
 * peaks.  Each function launches one kernel on `stream` (a hipStream_t,
 * NULL = default) and returns the bytes or flops that launch performs (the
 * caller times it, e.g. with HIP events), or a negative value on a bad
 * argument or launch error.  Device buffers are caller-owned; nothing is
 * allocated.  A workgroup has bcs_probe_threads_per_block() threads.
 */
#ifndef BCS_PROBE_H
#define BCS_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Threads per workgroup of every probe kernel (256). */
int bcs_probe_threads_per_block(void);

/* HBM stream: out[i] = in[i] for n FP64 words (n even; device buffers of n
 * doubles that do not overlap), `blocks` workgroups grid-striding.  Returns
 * 16 n (bytes read + written). */
double bcs_probe_copy(const double* in, double* out, int64_t n, int32_t blocks, void* stream);

/* LDS gathers: every thread reads 16 FP64 words from its workgroup's 32 KiB
 * LDS array per round, `rounds` rounds; pattern 0 = each wave reads 64
 * consecutive words per load (no bank conflicts), 1 = each lane reads a
 * pseudo-random word.  out: device FP64 [blocks * 256] (one sum per thread).
 * Returns the bytes gathered, 128 * rounds * 256 * blocks. */
double bcs_probe_lds(double* out, int64_t rounds, int32_t pattern, int32_t blocks, void* stream);

/* Vector FMA rate: 16 independent FMA chains per thread, `rounds` steps,
 * FP64 (fp64 = 1; out: device FP64 [blocks * 256]) or FP32 (fp64 = 0; out:
 * device FP32 [blocks * 256]; plain, not packed, FMAs).  Returns the flops,
 * 32 * rounds * 256 * blocks. */
double bcs_probe_fma(void* out, int64_t rounds, int32_t fp64, int32_t blocks, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* BCS_PROBE_H */
