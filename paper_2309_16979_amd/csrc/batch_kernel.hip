// Batched tile passes: one launch runs the same-level pass of many circuits
// (or parameter sets). Workgroup b finds its item by binary search in the
// launch's prefix table of tile counts, then runs that item's pass exactly as
// the single-circuit pass kernel does (decode -> ops -> encode on its tile).
#include <hip/hip_runtime.h>

#include "tile_ops.h"

namespace msv {

template <typename T, int TB>
__global__ __launch_bounds__(kThreads) void batch_pass_kernel(const BatchItem *__restrict__ items,
                                                              const uint64_t *__restrict__ prefix, int n_items)
{
    constexpr int TILE = 1 << TB;
    constexpr int NAB = TILE >> 6;
    constexpr int NSB = 2 * NAB;
    constexpr int NW = kThreads / 64;

    __shared__ T sre[TILE];
    __shared__ T sim[TILE];
    __shared__ uint64_t sG[NAB];
    __shared__ uint32_t sW[NSB];
    __shared__ int32_t sA[NSB];
    __shared__ uint32_t sOff[NSB];
    __shared__ double sred[2 * NW];
    __shared__ T sph[PhaseScratch<TB>::size];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // item: largest i with prefix[i] <= blockIdx.x
    const uint64_t bx = blockIdx.x;
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= bx) lo = mid;
        else hi = mid - 1;
    }
    const BatchItem &it = items[lo];
    const PassGeom &geo = it.geo;
    const PassBuffers &buf = it.buf;
    const uint64_t local = bx - prefix[lo];
    const uint64_t tile = geo.tile_begin + local;
    const uint64_t base = tile_base(geo, tile);
    tile_blocks<TB>(geo, base, sG);
    __syncthreads();
    tile_load<T, TB, true>(sre, sim, sG, buf.amps_in, buf.in, buf.step, buf.scale, wave, lane);
    __syncthreads();
    const T *pool = (const T *)buf.pool;
    for (int oi = 0; oi < geo.n_ops; ++oi) {
        const OpDesc op = buf.ops[geo.op_begin + oi];
        apply_op<T, TB>(sre, sim, op, pool + 2 * (int64_t)op.mat, base, geo.n, sph);
        __syncthreads();
    }
    double nrm = 0.0, err = 0.0;
    const uint64_t slot = (tile - buf.slot_tile0) * (uint64_t)(32 * NSB);
    const uint32_t words = tile_store<T, TB, true>(sre, sim, sG, sW, sA, sOff, buf.amps_out, buf.out, slot,
                                                   buf.inv_step, buf.step, buf.check_err, buf.flags, nrm, err, wave,
                                                   lane);
    nrm = wave_sum_f64(nrm);
    err = wave_max_f64(err);
    if (lane == 0) { sred[wave] = nrm; sred[NW + wave] = err; }
    __syncthreads();
    if (tid == 0 && buf.part) {
        double a = 0.0, e = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) { a += sred[w]; e = fmax(e, sred[NW + w]); }
        buf.part[3 * local] = a;
        buf.part[3 * local + 1] = e;
        buf.part[3 * local + 2] = (double)words;
    }
}

template <typename T, int TB>
static hipError_t batch_tb(const BatchItem *items, const uint64_t *prefix, int n_items, uint64_t total_tiles,
                           hipStream_t stream)
{
    hipLaunchKernelGGL((batch_pass_kernel<T, TB>), dim3((unsigned)total_tiles), dim3(kThreads), 0, stream, items,
                       prefix, n_items);
    return hipGetLastError();
}

template <typename T>
static hipError_t batch_t(int tb, const BatchItem *items, const uint64_t *prefix, int n_items, uint64_t total_tiles,
                          hipStream_t stream)
{
    switch (tb) {
    case 8: return batch_tb<T, 8>(items, prefix, n_items, total_tiles, stream);
    case 9: return batch_tb<T, 9>(items, prefix, n_items, total_tiles, stream);
    case 10: return batch_tb<T, 10>(items, prefix, n_items, total_tiles, stream);
    case 11: return batch_tb<T, 11>(items, prefix, n_items, total_tiles, stream);
    case 12: return batch_tb<T, 12>(items, prefix, n_items, total_tiles, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_pass(bool is_double, int tb, const BatchItem *items, const uint64_t *prefix, int n_items,
                             uint64_t total_tiles, hipStream_t stream)
{
    if (n_items <= 0 || total_tiles == 0) return hipSuccess;
    if (total_tiles > 0x7fffffffull) return hipErrorInvalidValue;
    return is_double ? batch_t<double>(tb, items, prefix, n_items, total_tiles, stream)
                     : batch_t<float>(tb, items, prefix, n_items, total_tiles, stream);
}

}  // namespace msv
