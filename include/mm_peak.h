/*
 * mm_peak.h -- measurement aid beside libmm (separate library, libmm_peak.so):
 * the matrix-core throughput a kernel doing nothing but MFMAs reaches on this
 * GPU, the ceiling against which the products' fraction of the datasheet
 * peak is read, and a probe of how matrix and vector instructions share a
 * SIMD.  It computes no product.
 */
#ifndef MM_PEAK_H
#define MM_PEAK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * mm_peak_mfma -- enqueue one launch of an MFMA-only kernel on `stream`
 * (hipStream_t, NULL = the null stream): `blocks` workgroups of 256 threads,
 * each wave running `iters` rounds of `chains` (8, 16 or 32) independent
 * accumulator chains of
 *   dtype 0: v_mfma_f64_16x16x4_f64   (2048 FLOP each)
 *   dtype 1: v_mfma_f32_16x16x4_f32   (2048 FLOP each)
 *   dtype 2: v_mfma_f32_16x16x32_bf16 (16384 FLOP each)
 * so the launch executes blocks * 4 * iters * chains MFMAs.  `out` (device,
 * blocks * 256 floats) receives one value per thread so nothing is optimised
 * away.  Returns 0, or -1 for a bad argument, -3 for a launch error.
 */
int32_t mm_peak_mfma(int32_t dtype, int32_t chains, int32_t blocks, int32_t iters, float *out, void *stream);

/*
 * mm_peak_overlap -- enqueue one launch that asks whether a SIMD overlaps
 * matrix instructions of some waves with vector instructions of others:
 * `blocks` workgroups of 512 threads; waves 0-3 of each run `iters` rounds of
 * 8 independent v_mfma_f32_16x16x32_bf16 chains, waves 4-7 `iters` rounds of
 * 64 FP32 fused multiply-adds over 16 independent chains.  role 0 runs both
 * kinds, 1 only the matrix waves, 2 only the vector waves (the others exit at
 * once).  With both kinds on every SIMD (blocks >= 2 per CU), role 0 taking
 * as long as roles 1 and 2 added means the SIMD issues them in turn; as long
 * as the longer, that it overlaps them.  `out` (device, blocks * 512 floats)
 * receives one value per thread.  Returns 0, or -1 for a bad argument, -3 for
 * a launch error.
 */
int32_t mm_peak_overlap(int32_t role, int32_t blocks, int32_t iters, float *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MM_PEAK_H */
