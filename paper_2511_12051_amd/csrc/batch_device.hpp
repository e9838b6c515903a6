// Persistent batched launches: one grid runs the blocks of several
// independent launches of the same kernel body (one per batch item).  Item k
// owns the flattened block range [starts[k], starts[k+1]); the grid strides
// over the whole range, so any number of items with uneven sizes share one
// launch whose size matches the machine rather than the work.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace plk {

template <typename Args>
struct BatchRange {
    const Args* __restrict__ items;   // per-item arguments (device memory)
    const int64_t* __restrict__ starts;  // n + 1 block offsets
    int n;
    int64_t total;
};

// item owning flattened block b (n is small: a linear scan of uniform values)
__device__ __forceinline__ int batch_item(const int64_t* __restrict__ starts, int n, int64_t b) {
    int k = 0;
    while (k + 1 < n && starts[k + 1] <= b) ++k;
    return k;
}

}  // namespace plk
