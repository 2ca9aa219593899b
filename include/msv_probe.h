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
 * streams (then *gbps counts the bytes of both directions), 3 device-to-host
 * with the copy kind hipMemcpyDeviceToDeviceNoCU (a copy engine, no compute
 * units; the pinned buffer is device-addressable). */
int msv_probe_host_link(size_t bytes, int direction, int reps, double *gbps);

/* Dense matrix-core throughput: 4 workgroups of 4 waves per compute unit,
 * each wave running independent accumulator chains of `iters` (>= 1) MFMA
 * ops, 3 launches after one warm-up, timed with HIP events.
 * precision (enum msv_mma): MSV_MMA_F64 v_mfma_f64_16x16x4f64 (8 chains),
 * MSV_MMA_F32 v_mfma_f32_16x16x4f32 (8 chains), MSV_MMA_BF16 the better of
 * v_mfma_f32_16x16x32_bf16 and v_mfma_f32_32x32x16_bf16 (4 chains).
 * *tflops = 2 M N K per op x ops / time / 1e12. */
int msv_probe_mfma_peak(int precision, int iters, double *tflops);

/* The paper's transfer experiment (Sec. 2, online stage step (2); Table 1):
 * moving a 2^n-amplitude complex128 state between host and GPU memory by
 *   MSV_XFER_SYNC           one synchronous hipMemcpy of the whole state;
 *   MSV_XFER_PER_AMPLITUDE  one hipMemcpyAsync of 16 bytes per amplitude on a
 *                           stream, as many calls as the state has amplitudes
 *                           (the paper's "async copy");
 *   MSV_XFER_STAGED_REMAP   one bulk copy into a device staging buffer, then a
 *                           GPU kernel that places every amplitude (the paper's
 *                           "buffer" strategy); device-to-host runs the kernel
 *                           first and the bulk copy second.
 * The remap places amplitude i of the host layout at device position
 * p(i) = ((i mod 2^h) << (n - h)) | (i >> h), h = n / 2 (the two halves of the
 * index bits exchanged: a chunked layout seen from the other side).
 * to_device: 1 host-to-device, 0 device-to-host; pinned: 1 hipHostMalloc'd
 * host buffer, 0 pageable (malloc'd). n_qubits in [6, 30]. The per-amplitude
 * strategy issues at most max_calls (>= 1) copies, of amplitudes spread over
 * the whole state, and extrapolates linearly; the others move everything.
 * Each measurement follows one untimed copy of the same kind.
 * *seconds = time of the whole-state transfer (extrapolated for the
 * per-amplitude strategy), *per_call = seconds per copy call issued,
 * *calls = copy calls issued. The data that arrives is checked against the
 * source (every amplitude, or every sampled one): MSV_E_STATE if any differs.
 * Allocates and frees its own buffers. */
enum msv_xfer_strategy { MSV_XFER_SYNC = 0, MSV_XFER_PER_AMPLITUDE = 1, MSV_XFER_STAGED_REMAP = 2 };
int msv_probe_transfer(int n_qubits, int strategy, int to_device, int pinned, size_t max_calls,
                       double *seconds, double *per_call, size_t *calls);

#ifdef __cplusplus
}
#endif
#endif /* MSV_PROBE_H_ */
