/*
 * gs_probe.h - measured issue rates of the GPU's FP32 arithmetic, for the
 * roofline that bounds the render kernels (their work is counted in VALU
 * lane-operations per in-cutoff pixel term, Eq. 7).
 */
#ifndef GS_PROBE_H
#define GS_PROBE_H

#include "gs.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Runs two short probe kernels on `stream` (about 1 s in all) on the current
 * device and returns, per second over the whole device: *fma_per_s, FP32
 * fused multiply-adds (v_fmac_f32, not packed: the library is built without
 * packed FP32) and *exp2_per_s, base-2 exponentials (v_exp_f32), each from
 * eight independent chains per lane with every SIMD holding eight waves (the
 * best of three timed launches).  Allocates a small device buffer and
 * synchronizes `stream`.  Both pointers are host memory and must not be NULL. */
GS_API gs_status gs_probe_alu(double *fma_per_s, double *exp2_per_s, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* GS_PROBE_H */
