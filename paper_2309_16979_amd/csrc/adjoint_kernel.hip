// Adjoint reverse sweep as tile passes over two states at once.
//
// For f = <psi_N| O |psi_N> with psi_N = U_N ... U_1 psi_0 and a gate
// U_k(theta) whose derivative is A_k U_k, df/dtheta = 2 Re <lambda_k| A_k |psi_k>
// with psi_k = U_k ... U_1 psi_0 and lambda_k = U_(k+1)^dagger ... U_N^dagger O psi_N.
// Walking the gates backwards, each workgroup keeps tiles of psi and lambda in
// LDS: at a probe op it adds its tile's share of <lambda| A |psi> to the
// probe's slot, at every other op it applies U^dagger to both tiles. Both
// states are decoded on load and re-encoded on store like any pass.
#include <hip/hip_runtime.h>

#include "persistent_queue.h"
#include "tile_ops.h"

namespace msv {

// One tile of a two-state pass: tile is the pass's tile index, pidx the
// index of its statistics triple in buf.psi.part / buf.lam.part. PRED: the
// stores may carry codec predictors other than 0, or the encode chooses them.
template <typename T, int TB, bool COMP, bool PRED>
__device__ __forceinline__ void adjoint_tile(const PassGeom &geo, const AdjointBuffers &buf, uint64_t tile,
                                             uint64_t pidx)
{
    constexpr int TILE = 1 << TB;
    constexpr int NAB = TILE >> 6;
    constexpr int NSB = 2 * NAB;
    constexpr int NW = kThreads / 64;

    __shared__ __attribute__((aligned(16))) T pre[TILE];
    __shared__ __attribute__((aligned(16))) T pim[TILE];
    __shared__ __attribute__((aligned(16))) T lre[TILE];
    __shared__ __attribute__((aligned(16))) T lim[TILE];
    __shared__ uint64_t sG[NAB];
    __shared__ uint32_t sW[NSB];
    __shared__ int32_t sA[NSB];
    __shared__ uint32_t sOff[NSB];
    __shared__ double sred[4 * NW];
    // phase-op tables during the ops, plane-word staging (128 words per
    // wave) during the decode
    constexpr int SX = (PhaseScratch<TB>::size * (int)sizeof(T) + 7) / 8 > 128 * NW
                           ? (PhaseScratch<TB>::size * (int)sizeof(T) + 7) / 8
                           : 128 * NW;
    __shared__ uint64_t sx[SX];
    T *const sph = reinterpret_cast<T *>(sx);

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint64_t base = tile_base(geo, tile);
    tile_blocks<TB>(geo, base, sG);
    __syncthreads();
    tile_load<T, TB, COMP, PRED>(pre, pim, sG, buf.psi.amps_in, buf.psi.in, buf.psi.step, 1.0, wave, lane,
                                 sx + 128 * wave);
    tile_load<T, TB, COMP, PRED>(lre, lim, sG, buf.lam.amps_in, buf.lam.in, buf.lam.step, 1.0, wave, lane,
                                 sx + 128 * wave);
    __syncthreads();

    const T *pool = (const T *)buf.psi.pool;
    for (int oi = 0; oi < geo.n_ops; ++oi) {
        const OpDesc op = load_op(buf.psi.ops + geo.op_begin + oi);
        const T *M = pool + 2 * (int64_t)op.mat;
        if (op.type == OP_GRAD) {
            double ar = 0.0, ai = 0.0;
            probe<T, TB>(pre, pim, lre, lim, op, M, base, ar, ai);
            ar = wave_sum_f64(ar);
            ai = wave_sum_f64(ai);
            if (lane == 0) { sred[wave] = ar; sred[NW + wave] = ai; }
            __syncthreads();
            if (tid == 0) {
                double sr = 0.0, si = 0.0;
#pragma unroll
                for (int w = 0; w < NW; ++w) { sr += sred[w]; si += sred[NW + w]; }
                const uint64_t at = 2 * ((uint64_t)op.slot * buf.grad_stride + tile);
                buf.grad_part[at] = sr;
                buf.grad_part[at + 1] = si;
            }
            __syncthreads();
        } else {
            apply_op<T, TB>(pre, pim, op, M, base, geo.n, sph);
            __syncthreads();
            apply_op<T, TB>(lre, lim, op, M, base, geo.n, sph);
            __syncthreads();
        }
    }

    const uint64_t slot = (tile - buf.psi.slot_tile0) * (uint64_t)(32 * NSB);
    double n1 = 0.0, e1 = 0.0, n2 = 0.0, e2 = 0.0;
    const uint32_t w1 = tile_store<T, TB, COMP, false, PRED>(pre, pim, sG, sW, sA, sOff, buf.psi.amps_out, buf.psi.out, slot,
                                                buf.psi.inv_step, buf.psi.step, buf.psi.check_err, buf.psi.pred_mode,
                                                buf.psi.flags, n1,
                                                e1, wave, lane);
    __syncthreads();
    const uint32_t w2 = tile_store<T, TB, COMP, false, PRED>(lre, lim, sG, sW, sA, sOff, buf.lam.amps_out, buf.lam.out, slot,
                                                buf.lam.inv_step, buf.lam.step, buf.lam.check_err, buf.lam.pred_mode,
                                                buf.lam.flags, n2,
                                                e2, wave, lane);
    n1 = wave_sum_f64(n1);
    e1 = wave_max_f64(e1);
    n2 = wave_sum_f64(n2);
    e2 = wave_max_f64(e2);
    if (lane == 0) {
        sred[wave] = n1;
        sred[NW + wave] = e1;
        sred[2 * NW + wave] = n2;
        sred[3 * NW + wave] = e2;
    }
    __syncthreads();
    if (tid == 0) {
        double a = 0.0, e = 0.0, b = 0.0, f = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            a += sred[w];
            e = fmax(e, sred[NW + w]);
            b += sred[2 * NW + w];
            f = fmax(f, sred[3 * NW + w]);
        }
        if (buf.psi.part) {
            buf.psi.part[3 * pidx] = a;
            buf.psi.part[3 * pidx + 1] = e;
            buf.psi.part[3 * pidx + 2] = (double)w1;
        }
        if (buf.lam.part) {
            buf.lam.part[3 * pidx] = b;
            buf.lam.part[3 * pidx + 1] = f;
            buf.lam.part[3 * pidx + 2] = (double)w2;
        }
    }
}

template <typename T, int TB, bool COMP, bool PRED>
__global__ __launch_bounds__(kThreads) void adjoint_kernel(PassGeom geo, AdjointBuffers buf)
{
    const uint32_t b = xcd_tile();
    adjoint_tile<T, TB, COMP, PRED>(geo, buf, geo.tile_begin + b, b);
}

// Every two-state pass of many parameter sets: (set, level, tile) items of
// the persistent queue.
template <typename T, int TB, bool COMP>
__global__ __launch_bounds__(kThreads) void adjoint_persistent_kernel(const AdjointDesc *__restrict__ descs,
                                                                      const uint64_t *__restrict__ prefix, int n_desc,
                                                                      uint64_t n_items, unsigned long long *head,
                                                                      unsigned int *done, uint32_t *flags,
                                                                      uint64_t spin_limit)
{
    run_queue(descs, prefix, n_desc, n_items, head, done, flags, spin_limit, [&](const AdjointDesc &d, uint64_t local) {
        adjoint_tile<T, TB, COMP, false>(d.geo, d.buf, d.geo.tile_begin + local, local);
    });
}

template <typename T, int TB, bool COMP>
static hipError_t adj_persistent_tb(const AdjointDesc *descs, const uint64_t *prefix, int n_desc, uint64_t n_items,
                                    unsigned long long *head, unsigned int *done, uint32_t *flags,
                                    uint64_t spin_limit, int *grid, hipStream_t stream)
{
    auto k = adjoint_persistent_kernel<T, TB, COMP>;
    *grid = occupancy_grid(k, n_items);
    hipLaunchKernelGGL(k, dim3((unsigned)*grid), dim3(kThreads), 0, stream, descs, prefix, n_desc, n_items, head, done,
                       flags, spin_limit);
    return hipGetLastError();
}

template <typename T, bool COMP>
static hipError_t adj_persistent_t(int tb, const AdjointDesc *descs, const uint64_t *prefix, int n_desc,
                                   uint64_t n_items, unsigned long long *head, unsigned int *done, uint32_t *flags,
                                   uint64_t spin_limit, int *grid, hipStream_t stream)
{
    switch (tb) {
    case 8: return adj_persistent_tb<T, 8, COMP>(descs, prefix, n_desc, n_items, head, done, flags, spin_limit, grid, stream);
    case 9: return adj_persistent_tb<T, 9, COMP>(descs, prefix, n_desc, n_items, head, done, flags, spin_limit, grid, stream);
    case 10: return adj_persistent_tb<T, 10, COMP>(descs, prefix, n_desc, n_items, head, done, flags, spin_limit, grid, stream);
    case 11: return adj_persistent_tb<T, 11, COMP>(descs, prefix, n_desc, n_items, head, done, flags, spin_limit, grid, stream);
    case 12: return adj_persistent_tb<T, 12, COMP>(descs, prefix, n_desc, n_items, head, done, flags, spin_limit, grid, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_adjoint_persistent(bool is_double, bool compressed, int tb, const AdjointDesc *descs,
                                     const uint64_t *prefix, int n_desc, uint64_t n_items, unsigned long long *head,
                                     unsigned int *done, uint32_t *flags, uint64_t spin_limit, int *grid,
                                     hipStream_t stream)
{
    *grid = 0;
    if (n_desc <= 0 || n_items == 0) return hipSuccess;
    if (is_double)
        return compressed ? adj_persistent_t<double, true>(tb, descs, prefix, n_desc, n_items, head, done, flags,
                                                           spin_limit, grid, stream)
                          : adj_persistent_t<double, false>(tb, descs, prefix, n_desc, n_items, head, done, flags,
                                                            spin_limit, grid, stream);
    return compressed ? adj_persistent_t<float, true>(tb, descs, prefix, n_desc, n_items, head, done, flags,
                                                      spin_limit, grid, stream)
                      : adj_persistent_t<float, false>(tb, descs, prefix, n_desc, n_items, head, done, flags,
                                                       spin_limit, grid, stream);
}

template <typename T, int TB>
static hipError_t adj_tb(bool comp, const PassGeom &geo, const AdjointBuffers &buf, hipStream_t stream)
{
    const dim3 grid((unsigned)geo.n_tiles), block(kThreads);
    const bool pred = buf.psi.pred_mode || buf.psi.in_pred || buf.lam.pred_mode || buf.lam.in_pred;
    if (comp && pred) hipLaunchKernelGGL((adjoint_kernel<T, TB, true, true>), grid, block, 0, stream, geo, buf);
    else if (comp) hipLaunchKernelGGL((adjoint_kernel<T, TB, true, false>), grid, block, 0, stream, geo, buf);
    else hipLaunchKernelGGL((adjoint_kernel<T, TB, false, false>), grid, block, 0, stream, geo, buf);
    return hipGetLastError();
}

template <typename T>
static hipError_t adj_t(bool comp, const PassGeom &geo, const AdjointBuffers &buf, hipStream_t stream)
{
    switch (geo.tb) {
    case 6: return adj_tb<T, 6>(comp, geo, buf, stream);
    case 7: return adj_tb<T, 7>(comp, geo, buf, stream);
    case 8: return adj_tb<T, 8>(comp, geo, buf, stream);
    case 9: return adj_tb<T, 9>(comp, geo, buf, stream);
    case 10: return adj_tb<T, 10>(comp, geo, buf, stream);
    case 11: return adj_tb<T, 11>(comp, geo, buf, stream);
    case 12: return adj_tb<T, 12>(comp, geo, buf, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_adjoint_pass(bool is_double, bool compressed, const PassGeom &geo, const AdjointBuffers &buf,
                               hipStream_t stream)
{
    if (geo.n_tiles == 0) return hipSuccess;
    if (geo.n_tiles > 0x7fffffffull) return hipErrorInvalidValue;
    return is_double ? adj_t<double>(compressed, geo, buf, stream) : adj_t<float>(compressed, geo, buf, stream);
}

// Slot blockIdx.x of set blockIdx.y (sets back to back: n_slots slots of
// stride tiles each).
__global__ __launch_bounds__(kThreads) void grad_reduce_kernel(const double *part, uint64_t stride, double *out)
{
    __shared__ double sr[kThreads], si[kThreads];
    const uint64_t s = blockIdx.x;
    part += 2 * (uint64_t)blockIdx.y * gridDim.x * stride;
    out += 2 * (uint64_t)blockIdx.y * gridDim.x;
    double a = 0.0, b = 0.0;
    for (uint64_t t = threadIdx.x; t < stride; t += kThreads) {
        a += part[2 * (s * stride + t)];
        b += part[2 * (s * stride + t) + 1];
    }
    sr[threadIdx.x] = a;
    si[threadIdx.x] = b;
    __syncthreads();
    for (int h = kThreads / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sr[threadIdx.x] += sr[threadIdx.x + h];
            si[threadIdx.x] += si[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[2 * s] = sr[0]; out[2 * s + 1] = si[0]; }
}

hipError_t launch_grad_reduce(const double *grad_part, uint64_t stride, int n_slots, double *out, hipStream_t stream)
{
    return launch_grad_reduce_multi(grad_part, stride, n_slots, 1, out, stream);
}

hipError_t launch_grad_reduce_multi(const double *grad_part, uint64_t stride, int n_slots, int n_sets, double *out,
                                    hipStream_t stream)
{
    if (n_slots <= 0 || n_sets <= 0) return hipSuccess;
    hipLaunchKernelGGL(grad_reduce_kernel, dim3((unsigned)n_slots, (unsigned)n_sets), dim3(kThreads), 0, stream,
                       grad_part, stride, out);
    return hipGetLastError();
}

}  // namespace msv
