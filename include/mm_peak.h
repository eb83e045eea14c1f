/*
 * mm_peak.h -- measurement aid beside libmm (separate library, libmm_peak.so):
 * the matrix-core throughput a kernel doing nothing but MFMAs reaches on this
 * GPU, the ceiling against which the products' fraction of the datasheet
 * peak is read.  It computes no product.
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

#ifdef __cplusplus
}
#endif

#endif /* MM_PEAK_H */
