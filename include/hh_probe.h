/*
 * hh_probe.h -- measurement utility of libhh (not part of the method).
 *
 * hh_probe_issue launches `blocks` blocks of 256 lanes; each lane runs 8
 * independent chains of `iters` operations of the chosen kind, i.e.
 * blocks * 256 * 8 * iters operations in total (twice that for
 * HH_PROBE_MIX, which interleaves an exp chain with an fma chain).  Timing the launch on
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
  HH_PROBE_MIX = 6    /* one v_exp_f32 and one v_fma_f32 chain per slot (2 ops) */
};

int32_t hh_probe_issue(int32_t op, int32_t iters, int32_t blocks, float* out, int32_t n_out,
                       void* stream);

#ifdef __cplusplus
}
#endif
#endif
