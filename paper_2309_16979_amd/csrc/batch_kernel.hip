// Persistent batched pass kernel: one launch runs every pass of many
// circuits (or parameter sets). Work items are (circuit, pass level, tile)
// triples in level-major order; workgroups take them from a device queue
// (atomic counter) and, before running a tile, wait until every tile of the
// circuit's previous levels has finished (per-circuit completion counters).
// Each tile runs exactly as in the single-circuit pass kernel (decode -> ops
// -> encode).
#include <hip/hip_runtime.h>

#include "pass_kernel.h"

namespace msv {

template <typename T, int TB, int KMAX>
__global__ __launch_bounds__(kThreads, (PassOccupancy<TB, KMAX>::waves)) void batch_persistent_kernel(
    const BatchDesc *__restrict__ descs, const uint64_t *__restrict__ prefix, int n_desc, uint64_t n_items,
    unsigned long long *head, unsigned int *done, uint32_t *flags, uint64_t spin_limit)
{
    __shared__ uint64_t s_item;
    __shared__ int s_go;
    const int tid = threadIdx.x;
    for (;;) {
        __syncthreads();   // the previous item's LDS is no longer read
        if (tid == 0) s_item = atomicAdd(head, 1ull);
        __syncthreads();
        const uint64_t item = s_item;
        if (item >= n_items) break;
        // descriptor: largest d with prefix[d] <= item
        int lo = 0, hi = n_desc - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= item) lo = mid;
            else hi = mid - 1;
        }
        const BatchDesc &d = descs[lo];
        if (tid == 0) {
            int go = 1;
            uint64_t spins = 0;
            while (__hip_atomic_load(done + d.circuit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < d.need) {
                if ((__hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kFlagQueueTimeout) ||
                    ++spins > spin_limit) {
                    atomicOr(flags, kFlagQueueTimeout);
                    go = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            // acquire: the earlier levels' stores are visible to this workgroup
            __threadfence();
            s_go = go;
        }
        __syncthreads();
        if (!s_go) break;
        const uint64_t local = item - prefix[lo];
        pass_tile<T, TB, true, true, KMAX, MMA_NONE, false>(d.geo, d.buf, d.geo.tile_begin + local, local);
        // release: every wave makes its own stores of the tile visible to the
        // whole device (consumers may run on another XCD, behind another L2)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (tid == 0) atomicAdd(done + d.circuit, 1u);
    }
}

template <typename K>
static int occupancy_grid(K kernel, uint64_t n_items)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kThreads, 0) != hipSuccess || per < 1) {
        (void)hipGetLastError();
        per = 1;
        if (cus < 1) cus = 1;
    }
    const uint64_t g = (uint64_t)cus * (uint64_t)per;
    return (int)(g < n_items ? g : n_items);
}

template <typename T, int TB>
static hipError_t batch_tb(int max_k, const BatchDesc *descs, const uint64_t *prefix, int n_desc, uint64_t n_items,
                           unsigned long long *head, unsigned int *done, uint32_t *flags, uint64_t spin_limit,
                           int *grid, hipStream_t stream)
{
    if (max_k <= 3) {
        auto k = batch_persistent_kernel<T, TB, 3>;
        *grid = occupancy_grid(k, n_items);
        hipLaunchKernelGGL(k, dim3((unsigned)*grid), dim3(kThreads), 0, stream, descs, prefix, n_desc, n_items, head,
                           done, flags, spin_limit);
    } else {
        auto k = batch_persistent_kernel<T, TB, 5>;
        *grid = occupancy_grid(k, n_items);
        hipLaunchKernelGGL(k, dim3((unsigned)*grid), dim3(kThreads), 0, stream, descs, prefix, n_desc, n_items, head,
                           done, flags, spin_limit);
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t batch_t(int tb, int max_k, const BatchDesc *descs, const uint64_t *prefix, int n_desc,
                          uint64_t n_items, unsigned long long *head, unsigned int *done, uint32_t *flags,
                          uint64_t spin_limit, int *grid, hipStream_t stream)
{
    switch (tb) {
    case 8: return batch_tb<T, 8>(max_k, descs, prefix, n_desc, n_items, head, done, flags, spin_limit, grid, stream);
    case 9: return batch_tb<T, 9>(max_k, descs, prefix, n_desc, n_items, head, done, flags, spin_limit, grid, stream);
    case 10: return batch_tb<T, 10>(max_k, descs, prefix, n_desc, n_items, head, done, flags, spin_limit, grid, stream);
    case 11: return batch_tb<T, 11>(max_k, descs, prefix, n_desc, n_items, head, done, flags, spin_limit, grid, stream);
    case 12: return batch_tb<T, 12>(max_k, descs, prefix, n_desc, n_items, head, done, flags, spin_limit, grid, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_persistent(bool is_double, int tb, int max_k, const BatchDesc *descs, const uint64_t *prefix,
                                   int n_desc, uint64_t n_items, unsigned long long *head, unsigned int *done,
                                   uint32_t *flags, uint64_t spin_limit, int *grid, hipStream_t stream)
{
    *grid = 0;
    if (n_desc <= 0 || n_items == 0) return hipSuccess;
    return is_double ? batch_t<double>(tb, max_k, descs, prefix, n_desc, n_items, head, done, flags, spin_limit, grid,
                                       stream)
                     : batch_t<float>(tb, max_k, descs, prefix, n_desc, n_items, head, done, flags, spin_limit, grid,
                                      stream);
}

}  // namespace msv
