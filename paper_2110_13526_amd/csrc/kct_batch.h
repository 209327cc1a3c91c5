// kct_batch.h -- device helpers of the batched kernels.
#pragma once

#include "kct_internal.h"

namespace kct {

// The instance that owns workgroup w of a batched grid: the largest i with
// off[i] <= w (off is ascending, count + 1 entries, off[0] = 0).
__device__ __forceinline__ int batch_find(const int64_t *__restrict__ off, int count, int64_t w)
{
    int lo = 0, hi = count;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= w) lo = mid;
        else hi = mid;
    }
    // the same instance in every lane (w is the workgroup's): keep the
    // instance's fields in scalar registers
    return __builtin_amdgcn_readfirstlane(lo);
}

// The next item of a persistent step's queue, the same in every thread of the
// workgroup.  Items are handed out in increasing order; every workgroup keeps
// taking items until it draws one beyond the last, so the queue always drains.
__device__ __forceinline__ int64_t batch_pop(BatchQueue *q)
{
    __shared__ unsigned s_item;
    __syncthreads();  // the previous item's readers are done with s_item
    if (__builtin_amdgcn_workitem_id_x() == 0) s_item = atomicAdd(&q->next, 1u);
    __syncthreads();
    return (int64_t)s_item;
}

// Leave a persistent step: the last workgroup to leave (every other one has
// drawn its final item) resets the queue for the next launch of the step.
__device__ __forceinline__ void batch_exit(BatchQueue *q)
{
    if (__builtin_amdgcn_workitem_id_x() == 0) {
        __threadfence();
        const unsigned n = atomicAdd(&q->exited, 1u);
        if (n == __builtin_amdgcn_grid_size_x() / __builtin_amdgcn_workgroup_size_x() - 1) {
            atomicExch(&q->next, 0u);
            atomicExch(&q->exited, 0u);
        }
    }
}

}  // namespace kct
