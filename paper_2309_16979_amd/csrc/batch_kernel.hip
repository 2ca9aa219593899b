// Batched tile passes: one launch runs the same-level pass of many circuits
// (or parameter sets). Workgroup b finds its item by binary search in the
// launch's prefix table of tile counts, then runs that item's pass exactly as
// the single-circuit pass kernel does (decode -> ops -> encode on its tile).
#include <hip/hip_runtime.h>

#include "pass_kernel.h"

namespace msv {

template <typename T, int TB, int KMAX>
__global__ __launch_bounds__(kThreads, (PassOccupancy<TB, KMAX>::waves)) void batch_pass_kernel(
    const BatchItem *__restrict__ items, const uint64_t *__restrict__ prefix, int n_items)
{
    // item: largest i with prefix[i] <= blockIdx.x
    const uint64_t bx = blockIdx.x;
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= bx) lo = mid;
        else hi = mid - 1;
    }
    const BatchItem &it = items[lo];
    const uint64_t local = bx - prefix[lo];
    pass_tile<T, TB, true, true, KMAX, MMA_NONE>(it.geo, it.buf, it.geo.tile_begin + local, local);
}

template <typename T, int TB>
static hipError_t batch_tb(int max_k, const BatchItem *items, const uint64_t *prefix, int n_items,
                           uint64_t total_tiles, hipStream_t stream)
{
    if (max_k <= 3)
        hipLaunchKernelGGL((batch_pass_kernel<T, TB, 3>), dim3((unsigned)total_tiles), dim3(kThreads), 0, stream,
                           items, prefix, n_items);
    else
        hipLaunchKernelGGL((batch_pass_kernel<T, TB, 5>), dim3((unsigned)total_tiles), dim3(kThreads), 0, stream,
                           items, prefix, n_items);
    return hipGetLastError();
}

template <typename T>
static hipError_t batch_t(int tb, int max_k, const BatchItem *items, const uint64_t *prefix, int n_items,
                          uint64_t total_tiles, hipStream_t stream)
{
    switch (tb) {
    case 8: return batch_tb<T, 8>(max_k, items, prefix, n_items, total_tiles, stream);
    case 9: return batch_tb<T, 9>(max_k, items, prefix, n_items, total_tiles, stream);
    case 10: return batch_tb<T, 10>(max_k, items, prefix, n_items, total_tiles, stream);
    case 11: return batch_tb<T, 11>(max_k, items, prefix, n_items, total_tiles, stream);
    case 12: return batch_tb<T, 12>(max_k, items, prefix, n_items, total_tiles, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_pass(bool is_double, int tb, int max_k, const BatchItem *items, const uint64_t *prefix,
                             int n_items, uint64_t total_tiles, hipStream_t stream)
{
    if (n_items <= 0 || total_tiles == 0) return hipSuccess;
    if (total_tiles > 0x7fffffffull) return hipErrorInvalidValue;
    return is_double ? batch_t<double>(tb, max_k, items, prefix, n_items, total_tiles, stream)
                     : batch_t<float>(tb, max_k, items, prefix, n_items, total_tiles, stream);
}

}  // namespace msv
