// Persistent batched pass kernel: one launch runs every pass of many
// circuits (or parameter sets). Work items are (circuit, pass level, tile)
// triples in level-major order, taken from the device queue of
// persistent_queue.h. Each tile runs exactly as in the single-circuit pass
// kernel (decode -> ops -> encode; COMP = false: plain amplitudes, updated in
// place or copied from amps_in to amps_out).
#include <hip/hip_runtime.h>

#include "pass_kernel.h"
#include "persistent_queue.h"

namespace msv {

template <typename T, int TB, int KMAX, bool COMP>
__global__ __launch_bounds__(kThreads, (PassOccupancy<TB, KMAX>::waves)) void batch_persistent_kernel(
    const BatchDesc *__restrict__ descs, const uint64_t *__restrict__ prefix, int n_desc, uint64_t n_items,
    unsigned long long *head, unsigned int *done, uint32_t *flags, uint64_t spin_limit)
{
    run_queue(descs, prefix, n_desc, n_items, head, done, flags, spin_limit, [&](const BatchDesc &d, uint64_t local) {
        pass_tile<T, TB, COMP, COMP, KMAX, MMA_NONE, false, false>(d.geo, d.buf, d.geo.tile_begin + local, local);
    });
}

template <typename T, int TB, bool COMP>
static hipError_t batch_tb(int max_k, const BatchDesc *descs, const uint64_t *prefix, int n_desc, uint64_t n_items,
                           unsigned long long *head, unsigned int *done, uint32_t *flags, uint64_t spin_limit,
                           int *grid, hipStream_t stream)
{
    if (max_k <= 3) {
        auto k = batch_persistent_kernel<T, TB, 3, COMP>;
        *grid = occupancy_grid(k, n_items);
        hipLaunchKernelGGL(k, dim3((unsigned)*grid), dim3(kThreads), 0, stream, descs, prefix, n_desc, n_items, head,
                           done, flags, spin_limit);
    } else {
        auto k = batch_persistent_kernel<T, TB, 5, COMP>;
        *grid = occupancy_grid(k, n_items);
        hipLaunchKernelGGL(k, dim3((unsigned)*grid), dim3(kThreads), 0, stream, descs, prefix, n_desc, n_items, head,
                           done, flags, spin_limit);
    }
    return hipGetLastError();
}

template <typename T, bool COMP>
static hipError_t batch_t(int tb, int max_k, const BatchDesc *descs, const uint64_t *prefix, int n_desc,
                          uint64_t n_items, unsigned long long *head, unsigned int *done, uint32_t *flags,
                          uint64_t spin_limit, int *grid, hipStream_t stream)
{
    switch (tb) {
    case 8: return batch_tb<T, 8, COMP>(max_k, descs, prefix, n_desc, n_items, head, done, flags, spin_limit, grid, stream);
    case 9: return batch_tb<T, 9, COMP>(max_k, descs, prefix, n_desc, n_items, head, done, flags, spin_limit, grid, stream);
    case 10: return batch_tb<T, 10, COMP>(max_k, descs, prefix, n_desc, n_items, head, done, flags, spin_limit, grid, stream);
    case 11: return batch_tb<T, 11, COMP>(max_k, descs, prefix, n_desc, n_items, head, done, flags, spin_limit, grid, stream);
    case 12: return batch_tb<T, 12, COMP>(max_k, descs, prefix, n_desc, n_items, head, done, flags, spin_limit, grid, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_persistent(bool is_double, bool compressed, int tb, int max_k, const BatchDesc *descs,
                                   const uint64_t *prefix, int n_desc, uint64_t n_items, unsigned long long *head,
                                   unsigned int *done, uint32_t *flags, uint64_t spin_limit, int *grid,
                                   hipStream_t stream)
{
    *grid = 0;
    if (n_desc <= 0 || n_items == 0) return hipSuccess;
    if (is_double)
        return compressed ? batch_t<double, true>(tb, max_k, descs, prefix, n_desc, n_items, head, done, flags,
                                                  spin_limit, grid, stream)
                          : batch_t<double, false>(tb, max_k, descs, prefix, n_desc, n_items, head, done, flags,
                                                   spin_limit, grid, stream);
    return compressed ? batch_t<float, true>(tb, max_k, descs, prefix, n_desc, n_items, head, done, flags, spin_limit,
                                             grid, stream)
                      : batch_t<float, false>(tb, max_k, descs, prefix, n_desc, n_items, head, done, flags,
                                              spin_limit, grid, stream);
}

}  // namespace msv
