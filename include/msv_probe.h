/*
 * msv_probe.h - measured roofline denominators on the current HIP device.
 *
 * The throughput of the compressed pass is reported as a fraction of what the
 * hardware delivers: HBM bandwidth (the pass streams chunk bytes through it),
 * the host link (the host-store form streams compressed chunks between pinned
 * host memory and the GPU, the transfer the paper's Table 1 measures), and the
 * matrix cores (fused k-qubit unitaries as GEMMs). These calls measure each on
 * the current device. They allocate their own buffers (hipMalloc /
 * hipHostMalloc), free them before returning, and use streams of their own.
 *
 * Every function returns MSV_OK (0), MSV_E_ARG for an invalid argument, or
 * MSV_E_DEVICE when a HIP call fails (the message of msv_last_error is not
 * set by these calls).
 */
#ifndef MSV_PROBE_H_
#define MSV_PROBE_H_

#include <stddef.h>

#include "msv.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Device-to-device copy of `bytes` (>= 4096, rounded down to 16) by streaming
 * kernels with 16-byte loads and stores, `reps` (>= 1) times after one
 * warm-up per launch shape, timed with HIP events; the best of six shapes
 * (grid-stride with one load in flight, grid-stride with four non-temporal
 * loads in flight, one contiguous range per workgroup; 4 to 128 workgroups
 * of 256 threads per compute unit).
 * *gbps = 2 * bytes * reps / time / 1e9 (bytes read plus bytes written). */
int msv_probe_hbm_copy(size_t bytes, int reps, double *gbps);

/* Copies of `bytes` (>= 4096) between a pinned host buffer (hipHostMalloc)
 * and device memory with hipMemcpyAsync, `reps` (>= 1) times after one
 * warm-up, timed on the host around the synchronised copies.
 * direction: 0 host-to-device, 1 device-to-host, 2 both at once on two
 * streams (then *gbps counts the bytes of both directions). */
int msv_probe_host_link(size_t bytes, int direction, int reps, double *gbps);

/* Dense matrix-core throughput: 4 workgroups of 4 waves per compute unit,
 * each wave running independent accumulator chains of `iters` (>= 1) MFMA
 * ops, 3 launches after one warm-up, timed with HIP events.
 * precision (enum msv_mma): MSV_MMA_F64 v_mfma_f64_16x16x4f64 (8 chains),
 * MSV_MMA_F32 v_mfma_f32_16x16x4f32 (8 chains), MSV_MMA_BF16 the better of
 * v_mfma_f32_16x16x32_bf16 and v_mfma_f32_32x32x16_bf16 (4 chains).
 * *tflops = 2 M N K per op x ops / time / 1e12. */
int msv_probe_mfma_peak(int precision, int iters, double *tflops);

#ifdef __cplusplus
}
#endif
#endif /* MSV_PROBE_H_ */
