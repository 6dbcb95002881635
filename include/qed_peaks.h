/*
 * qed_peaks.h -- measured peaks of one MI355X (gfx950) for the roofline figures.
 *
 * Three microbenchmarks give the rates the generator's kernels are quoted against,
 * beside the published ones: the HBM bandwidth a plain stream can reach, and the
 * issue rate of non-packed FP32 and of FP64 fused multiply-adds (the library is
 * built without packed FP32 instructions, so the non-packed rate is the FP32 vector
 * ceiling its kernels can reach).  Not part of the generator's path.
 *
 * All pointers are DEVICE pointers owned by the caller; work is enqueued on
 * `stream` (a hipStream_t, NULL for the default stream) and each call waits for it.
 * Return value: 0 on success, -1 for a bad argument (nothing enqueued), -4 if a HIP
 * runtime call failed (the values of qed_status).
 */
#ifndef QED_PEAKS_H
#define QED_PEAKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QED_PEAKS_API __attribute__((visibility("default")))

/* Copy `bytes` (a multiple of 16, src and dst 16-byte aligned, not overlapping) from
 * src to dst `reps` times with 16-byte vector loads and stores, one element per
 * thread over a grid covering the buffer; *ms = mean milliseconds per copy (HIP
 * events on `stream`).  HBM rate: 2 * bytes / (*ms * 1e-3). */
QED_PEAKS_API int qed_peak_copy(const void *src, void *dst, uint64_t bytes, int reps, void *stream, float *ms);

/* Fused multiply-adds in registers: `blocks` blocks of 256 threads, each thread
 * running 8 independent chains for `iters` x 16 steps; dtype 0 = float (non-packed
 * v_fma_f32), 1 = double (v_fma_f64).  sink: blocks * 256 elements of that type,
 * written once (keeps the chains live).  *ms = milliseconds of the launch;
 * *flops = 2 * 8 * 16 * iters * blocks * 256. */
QED_PEAKS_API int qed_peak_fma(int dtype, void *sink, int blocks, uint64_t iters, void *stream, float *ms,
                               double *flops);

#ifdef __cplusplus
}
#endif
#endif
