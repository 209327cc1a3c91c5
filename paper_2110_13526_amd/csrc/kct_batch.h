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

}  // namespace kct
