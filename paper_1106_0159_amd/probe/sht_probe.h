/*
 * sht_probe.h -- throughput probes for the roofline of the benchmark,
 * libsht_probe.so (built beside, not into, the transform library libsht.so;
 * not part of the transform API).  They measure what one MI355X
 * (gfx950) attains on the instruction kinds the transform kernels use, with
 * no memory traffic in the timed loop: the benchmark reports its roofline
 * fractions against the nominal peaks and these measured rates beside them.
 * Callers: bench.py (--peak-probe).
 */
#ifndef SHT_PROBE_H
#define SHT_PROBE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Probe kinds:
 *   0  FP64 FMA on the vector ALUs (v_fma_f64), 8 independent chains per lane
 *   1  FP32 matrix instruction v_mfma_f32_16x16x4_f32, 8 independent accumulators per wave
 *   2  BF16 matrix instruction v_mfma_f32_16x16x32_bf16, 8 independent accumulators per wave
 *   3  kinds 1 and 0 interleaved: per iteration 8 FP32 matrix instructions and
 *      64 FP64 FMAs per lane (the work of kind 1 at the same iters plus kind 0
 *      at 8 x iters), to time whether vector and matrix work overlap
 * Workgroups of 256 threads. */
enum sht_probe_kind {
    SHT_PROBE_FMA_F64 = 0,
    SHT_PROBE_MFMA_F32 = 1,
    SHT_PROBE_MFMA_BF16 = 2,
    SHT_PROBE_MFMA_F32_FMA_F64 = 3
};

/* Floating-point operations one sht_probe_run with these arguments performs
 * (an FMA counts 2); 0 for invalid arguments (unknown kind, blocks or iters
 * below 1). */
double sht_probe_flops(int kind, int blocks, int iters);

/* Enqueues one probe launch on `stream` (a hipStream_t; NULL = the null
 * stream) and returns without waiting.
 *   out  DEVICE buffer of at least blocks * 256 * 8 bytes, written with one
 *        value per thread so that the work is not optimised away
 * Returns 0, -1 (invalid arguments, nothing enqueued) or -3 (the launch
 * failed). */
int sht_probe_run(int kind, int blocks, int iters, void *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SHT_PROBE_H */
