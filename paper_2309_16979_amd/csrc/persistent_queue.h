// Work queue of the persistent batched launches (many circuits, or many
// parameter sets of one circuit, in one launch).
//
// A work item is a group of d.group consecutive tiles (the last group of a
// descriptor may be shorter) of one descriptor d = (state, pass level).
// Items are numbered level-major: item i belongs to descriptor d with
// prefix[d] <= i < prefix[d + 1]. Workgroups take items in order from an
// atomic counter and, before running one, wait until every tile of the
// state's earlier levels has finished (per-state tile counters: d may start
// once done[d.circuit] >= d.need). Items only wait on items taken before
// them, so the queue always drains; a wait longer than spin_limit polls sets
// kFlagQueueTimeout and every workgroup then leaves the queue.
//
// Cross-XCD visibility costs an L2 write-back on release and an L2
// invalidate on acquire (agent scope), so tiles are grouped to pay them once
// per group, and the first level of a state (need = 0, inputs written before
// the launch) skips the acquire.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace msv {

template <typename Desc, typename Body>
__device__ __forceinline__ void run_queue(const Desc *__restrict__ descs, const uint64_t *__restrict__ prefix,
                                          int n_desc, uint64_t n_items, unsigned long long *head, unsigned int *done,
                                          uint32_t *flags, uint64_t spin_limit, Body &&body)
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
        const Desc &d = descs[lo];
        if (tid == 0) {
            int go = 1;
            if (d.need) {
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
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            s_go = go;
        }
        __syncthreads();
        if (!s_go) break;
        const uint64_t t0 = (item - prefix[lo]) * (uint64_t)d.group;
        const uint64_t t1 = t0 + d.group < d.geo.n_tiles ? t0 + d.group : d.geo.n_tiles;
        for (uint64_t t = t0; t < t1; ++t) {
            if (t != t0) __syncthreads();   // the previous tile's LDS is no longer read
            body(d, t);
        }
        // release: every wave makes its own stores of the group visible to
        // the whole device (consumers may run on another XCD, behind another L2)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (tid == 0) atomicAdd(done + d.circuit, (unsigned int)(t1 - t0));
    }
}

// Workgroups of a persistent launch: as many as fit on the device at once,
// at most the item count.
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

}  // namespace msv
