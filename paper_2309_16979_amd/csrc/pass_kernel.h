// The fused streamed pass: load (decode) -> apply every op of the pass in LDS
// -> store (encode), one workgroup per tile of 2^TB amplitudes.
//
// A pass (one stage of the paper's online loop, Sec. 2) is a run of gates whose
// non-diagonal qubits all fit into one tile: the tile's first six bits are
// qubits 0..5 (so it consists of whole 64-amplitude codec blocks) and its other
// TB-6 bits are the pass's qubits, which may lie inside a chunk or cross chunks
// (then the workgroup gathers blocks from 2^h chunks: the chunk-pair exchange).
// Every workgroup decodes its blocks into LDS (planar re / im), runs the op
// list with a barrier between ops, and re-encodes its blocks. Encoded payload
// goes to the workgroup's own heap slot (worst case 32 words per block), so
// no cross-workgroup scan is needed; W / A / OFF record where each block went.
#pragma once
#include <hip/hip_runtime.h>

#include "mfma_ops.h"
#include "reg_ops.h"
#include "tile_ops.h"

namespace msv {

// One tile of a pass: decode -> ops -> encode, then the workgroup's FP64
// statistics into part[3 pidx ..]. Shared by the single-state pass kernel and
// the batched kernel.
// XP: the codec's half-wave bit transposes (off in the persistent batch
// kernel, whose queue state leaves fewer registers for them).
template <typename T, int TB, bool LOADC, bool STOREC, int KMAX, int MF, bool PRED, bool XP = true>
__device__ __forceinline__ void pass_tile(const PassGeom &geo, const PassBuffers &buf, uint64_t tile, uint64_t pidx)
{
    constexpr int TILE = 1 << TB;
    constexpr int NAB = TILE >> 6;   // 64-amplitude blocks per tile
    constexpr int NSB = 2 * NAB;     // stream blocks (re + im planes)
    constexpr int NW = kThreads / 64;

    __shared__ __attribute__((aligned(16))) T samp[2 * TILE];   // re plane, then im plane
    T *const sre = samp, *const sim = samp + TILE;
    __shared__ uint64_t sG[NAB];
    __shared__ uint32_t sW[NSB];
    __shared__ int32_t sA[NSB];
    __shared__ uint32_t sOff[NSB];
    __shared__ double sred[3 * NW];
    // phase-op tables during the ops; per wave, 128 words of plane-word
    // staging during the decode and payload offsets during the encode
    constexpr int SX = (PhaseScratch<TB>::size * (int)sizeof(T) + 7) / 8 > 128 * NW
                           ? (PhaseScratch<TB>::size * (int)sizeof(T) + 7) / 8
                           : 128 * NW;
    __shared__ uint64_t sx[SX];
    T *const sph = reinterpret_cast<T *>(sx);

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform for the compiler
    const uint64_t base = tile_base(geo, tile);
    tile_blocks<TB>(geo, base, sG);
    __syncthreads();

    const double sc = buf.scale_src ? 1.0 / __builtin_sqrt(*buf.scale_src) : buf.scale;
    tile_load<T, TB, LOADC, PRED, XP>(sre, sim, sG, buf.amps_in, buf.in, buf.step, sc, wave, lane, sx + 128 * wave);
    __syncthreads();

    const T *pool = (const T *)buf.pool;
    for (int oi = 0; oi < geo.n_ops; ++oi) {
        const OpDesc op = load_op(buf.ops + geo.op_begin + oi);
        if (op.type == OP_SEG) {
            if constexpr (TB >= 10 && TB <= 13)
                run_segment<T, TB>(samp, op, buf.ops + geo.op_begin + oi + 1, pool, base, tile);
            oi += op.k;
        } else if (op.type == OP_OBS)
            op_obs<T, TB>(sre, sim, sG, buf.obs_masks, buf.obs_coeffs, buf.obs_terms);
        else if (MF != MMA_NONE && op.type == OP_MFMA)
            apply_mfma<T, TB, MF>(samp, op, pool + 2 * (int64_t)op.mat, base, wave, lane);
        else
            apply_op<T, TB, KMAX>(sre, sim, op, pool + 2 * (int64_t)op.mat, base, geo.n, sph);
        __syncthreads();
    }

    if (geo.out_perm) {
        // the output order moves whole blocks: block index bit i (qubit i + 6)
        // goes to qubit out_q[i + 6]
        for (int jb = tid; jb < NAB; jb += kThreads) {
            const uint64_t G = sG[jb];
            uint64_t o = 0;
            for (int i = 0; i < geo.n - 6; ++i) o |= ((G >> i) & 1ull) << (geo.out_q[i + 6] - 6);
            sG[jb] = o;
        }
        __syncthreads();
    }

    // the expectation of the stored state, when the caller asks for it with
    // this (last) pass; the store below overwrites the tile's values
    double ex = 0.0;
    if (buf.exp_part)
        ex = wave_sum_f64(tile_expect<T, TB, STOREC>(sre, sim, sG, buf.obs_masks, buf.obs_coeffs, buf.obs_terms,
                                                       buf.inv_step, buf.step, wave, lane));
    double nrm = 0.0, err = 0.0;
    const uint64_t slot = (tile - buf.slot_tile0) * (uint64_t)(32 * NSB);
    static_assert(NSB <= 256, "per-wave offsets hold 256 words");
    const uint32_t words = tile_store<T, TB, STOREC, true, PRED, XP>(sre, sim, sG, sW, sA, sOff, buf.amps_out, buf.out, slot,
                                                           buf.inv_step, buf.step, buf.check_err, buf.pred_mode, buf.flags, nrm,
                                                           err, wave, lane,
                                                           reinterpret_cast<uint32_t *>(sx + 128 * wave));
    // per-workgroup statistics (fixed reduction order)
    nrm = wave_sum_f64(nrm);
    err = wave_max_f64(err);
    if (lane == 0) { sred[wave] = nrm; sred[NW + wave] = err; sred[2 * NW + wave] = ex; }
    __syncthreads();
    if (tid == 0 && buf.part) {
        double a = 0.0, e = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) { a += sred[w]; e = fmax(e, sred[NW + w]); }
        buf.part[3 * pidx] = a;
        buf.part[3 * pidx + 1] = e;
        buf.part[3 * pidx + 2] = (double)words;
    }
    if (tid == 0 && buf.exp_part) {
        double x = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) x += sred[2 * NW + w];
        buf.exp_part[4 * pidx] = 0.0;
        buf.exp_part[4 * pidx + 1] = x;
        buf.exp_part[4 * pidx + 2] = 0.0;
        buf.exp_part[4 * pidx + 3] = 0.0;
    }
}

// Register cap: four waves per SIMD for the common variants (LDS allows four
// workgroups of 2^12 complex64 amplitudes per CU), two for the rest.
template <int TB, int KMAX> struct PassOccupancy { static constexpr int waves = (KMAX <= 3 && TB <= 12) ? 4 : 2; };

// PRED: the decode reads predictor ids and the encode carries predictor mode 1
// (buf.pred_mode). Variants without it assume predictor 0 throughout and are
// launched only when buf.pred_mode and buf.in_pred are both 0.
template <typename T, int TB, bool LOADC, bool STOREC, int KMAX, int MF, bool PRED>
__global__ __launch_bounds__(kThreads, (PassOccupancy<TB, KMAX>::waves)) void pass_kernel(PassGeom geo, PassBuffers buf)
{
    const uint32_t b = xcd_tile();
    pass_tile<T, TB, LOADC, STOREC, KMAX, MF, PRED>(geo, buf, geo.tile_begin + b, b);
}

template <typename T, int TB, int KMAX, int MF>
static hipError_t launch_k(bool load_c, bool store_c, const PassGeom &geo, const PassBuffers &buf,
                           hipStream_t stream)
{
    const dim3 grid((unsigned)geo.n_tiles), block(kThreads);
    const bool pred = (store_c && buf.pred_mode != 0) || (load_c && buf.in_pred != 0);
    if (load_c && store_c && pred)
        hipLaunchKernelGGL((pass_kernel<T, TB, true, true, KMAX, MF, true>), grid, block, 0, stream, geo, buf);
    else if (load_c && store_c)
        hipLaunchKernelGGL((pass_kernel<T, TB, true, true, KMAX, MF, false>), grid, block, 0, stream, geo, buf);
    else if (load_c && pred)
        hipLaunchKernelGGL((pass_kernel<T, TB, true, false, KMAX, MF, true>), grid, block, 0, stream, geo, buf);
    else if (load_c)
        hipLaunchKernelGGL((pass_kernel<T, TB, true, false, KMAX, MF, false>), grid, block, 0, stream, geo, buf);
    else if (store_c && pred)
        hipLaunchKernelGGL((pass_kernel<T, TB, false, true, KMAX, MF, true>), grid, block, 0, stream, geo, buf);
    else if (store_c)
        hipLaunchKernelGGL((pass_kernel<T, TB, false, true, KMAX, MF, false>), grid, block, 0, stream, geo, buf);
    else
        hipLaunchKernelGGL((pass_kernel<T, TB, false, false, KMAX, MF, false>), grid, block, 0, stream, geo, buf);
    return hipGetLastError();
}

// Passes whose VALU dense ops are at most 3 qubits wide run a variant compiled
// without the 4- and 5-qubit paths (fewer registers, higher occupancy). Passes
// with matrix-core ops run a variant that carries the MFMA path (tiles of at
// least 2^7 amplitudes, so that an op has 16 columns).
template <typename T, int TB, int MF>
static hipError_t launch_tb(bool load_c, bool store_c, const PassGeom &geo, const PassBuffers &buf,
                            hipStream_t stream)
{
    if constexpr (MF != MMA_NONE && TB < 7) {
        return hipErrorInvalidValue;
    } else {
        if (geo.max_k <= 3) return launch_k<T, TB, 3, MF>(load_c, store_c, geo, buf, stream);
        return launch_k<T, TB, 5, MF>(load_c, store_c, geo, buf, stream);
    }
}

// All tile sizes of one (type, matrix-core mode) variant; each variant is
// compiled in a translation unit of its own.
template <typename T, int MF>
hipError_t launch_pass_variant(bool load_c, bool store_c, const PassGeom &geo, const PassBuffers &buf,
                               hipStream_t stream)
{
    switch (geo.tb) {
    case 6: return launch_tb<T, 6, MF>(load_c, store_c, geo, buf, stream);
    case 7: return launch_tb<T, 7, MF>(load_c, store_c, geo, buf, stream);
    case 8: return launch_tb<T, 8, MF>(load_c, store_c, geo, buf, stream);
    case 9: return launch_tb<T, 9, MF>(load_c, store_c, geo, buf, stream);
    case 10: return launch_tb<T, 10, MF>(load_c, store_c, geo, buf, stream);
    case 11: return launch_tb<T, 11, MF>(load_c, store_c, geo, buf, stream);
    case 12: return launch_tb<T, 12, MF>(load_c, store_c, geo, buf, stream);
    case 13: return launch_tb<T, 13, MF>(load_c, store_c, geo, buf, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace msv
