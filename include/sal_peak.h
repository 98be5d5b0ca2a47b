/*
 * sal_peak.h -- microbenchmarks of the device's own throughput peaks, the
 * denominators of the roofline fractions that the benchmark reports next to the
 * published ones (matrix-core, vector-ALU and HBM rates as this device sustains
 * them).  Measurement aids only: no step of the saliency method uses them.
 *
 * Conventions as in sal.h: every pointer is caller-owned device memory of the
 * current HIP device, all work is enqueued on `stream` (time it with events on
 * that stream), arguments are checked on the host before anything is launched,
 * and sal_last_error() explains a non-zero status.
 */
#ifndef SAL_PEAK_H
#define SAL_PEAK_H

#include <stdint.h>

#include "sal.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SAL_PEAK_MFMA_F32 = 0,   /* v_mfma_f32_16x16x4_f32: 2,048 flops per wave instruction */
    SAL_PEAK_MFMA_BF16 = 1,  /* v_mfma_f32_32x32x16_bf16: 32,768 flops (the rate of 16x16x32) */
    SAL_PEAK_MFMA_F16 = 2,   /* v_mfma_f32_32x32x16_f16: 32,768 flops */
    SAL_PEAK_VALU_F32 = 3    /* v_fma_f32, one lane operation (2 flops) per lane */
} sal_peak_kind;

/* Flops of one sal_peak_compute launch (0 if an argument is out of range). */
int64_t sal_peak_compute_flops(int kind, int64_t iters, int64_t blocks);

/* Issues `iters` rounds of independent dependency chains of the instruction
 * `kind` names (4 chains of a matrix-core form, 8 of v_fma_f32), with every
 * operand 1, in each wave of `blocks` workgroups of 256 threads (4 waves).  out:
 * device float [blocks * 256]; thread i of the grid writes the sum of its
 * accumulators, which is exact and has a closed form: 64 * iters (MFMA_F32: 4
 * chains x 4 accumulators x K = 4), 1024 * iters (MFMA_BF16, MFMA_F16: 4 chains
 * x 16 accumulators x K = 16), 8 * iters (VALU_F32).
 * Limits: 1 <= iters <= 16384 (keeps every sum an exact float), 1 <= blocks <=
 * 2^20.  SAL_ERR_ARG otherwise. */
sal_status sal_peak_compute(int kind, int64_t iters, int64_t blocks, float* out, sal_stream stream);

/* HBM streaming over `bytes` (a positive multiple of 16; src and dst 16-byte
 * aligned) with `blocks` workgroups of 256 threads striding over 16-byte words.
 * kind 0 (read): reads src; thread i writes the sum of the floats it read to
 * out[i] (device float [blocks * 256]; dst unused).  kind 1 (copy): dst = src
 * (out unused; the ranges must not overlap).  1 <= blocks <= 2^20; SAL_ERR_ARG
 * otherwise. */
sal_status sal_peak_stream(int kind, const void* src, void* dst, int64_t bytes, float* out, int64_t blocks,
                           sal_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* SAL_PEAK_H */
