/*
 * hh_probe.h -- measurement utility of libhh (not part of the method).
 *
 * hh_probe_issue launches `blocks` blocks of 256 lanes; each lane runs 8
 * independent chains of `iters` operations of the chosen kind, i.e.
 * blocks * 256 * 8 * iters operations in total (twice that for
 * HH_PROBE_MIX, which interleaves an exp chain with an fma chain, and for
 * HH_PROBE_PKFMA16, whose instructions each do two).  The matrix probes run
 * blocks * 4 * iters * 2 products of 32x32x16 (32,768 flops each), the
 * second with 32 FMAs per lane interleaved, which shows whether matrix and
 * vector work overlap.  Timing the launch on
 * `stream` gives the chip's issue rate for that kind of operation, which
 * sets the denominators of the arithmetic roofline.  out: device float
 * [n_out] (written for the first n_out lanes).  Returns 0, -1 for bad
 * arguments, -3 for a launch error.
 */
#ifndef HH_PROBE_H
#define HH_PROBE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HH_PROBE_FMA = 0,   /* v_fma_f32 */
  HH_PROBE_EXP2 = 1,  /* v_exp_f32 */
  HH_PROBE_RCP = 2,   /* v_rcp_f32 */
  HH_PROBE_SQRT = 3,  /* v_sqrt_f32 */
  HH_PROBE_SIN = 4,   /* v_sin_f32 */
  HH_PROBE_MUL64 = 5, /* 32 x 32 -> 64-bit integer multiply */
  HH_PROBE_MIX = 6,   /* one v_exp_f32 and one v_fma_f32 chain per slot (2 ops) */
  HH_PROBE_PKFMA16 = 7, /* packed half-precision FMA (2 ops per instruction) */
  HH_PROBE_EXP16 = 8,   /* v_exp_f16 */
  HH_PROBE_MFMA16 = 9,  /* 2 chains of 32x32x16 f16 matrix products per iteration and wavefront */
  HH_PROBE_MFMA16_VALU = 10 /* the same plus 32 FP32 FMAs per lane and iteration */
};

int32_t hh_probe_issue(int32_t op, int32_t iters, int32_t blocks, float* out, int32_t n_out,
                       void* stream);

/* Barrier floor of the persistent network kernel: a cooperative launch of
 * `blocks` blocks of the network kernel's size runs `steps` grid barriers
 * (mode 0), or each barrier followed by the two per-neuron accumulator
 * read-and-clear atomics the network step performs (mode 1), or the
 * flag-array barrier alone (mode 2: each block stores its arrival in a slot
 * of its own, one wavefront gathers them and releases the grid).  Timing it on
 * `stream` gives the synchronization cost per step with no neuron or
 * synapse work.  work: device scratch of hh_probe_barrier_bytes(blocks)
 * bytes (zeroed by the call).  Returns 0, -1 for bad arguments, -2 for a
 * short work buffer, -3 for a launch error, -5 if the blocks cannot all be
 * resident at once. */
size_t hh_probe_barrier_bytes(int32_t blocks);
int32_t hh_probe_barrier(int32_t steps, int32_t blocks, int32_t mode, void* work, size_t work_bytes,
                         void* stream);

#ifdef __cplusplus
}
#endif
#endif
