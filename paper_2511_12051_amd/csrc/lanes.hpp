// Lane-level helpers shared by the device code: the workgroup size of the
// one-thread-per-item stages, the lane index and the wavefront fence.
#pragma once
#include <hip/hip_runtime.h>

namespace plk {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0));
}

// Orders this wavefront's LDS stores before its later LDS loads of words
// that other lanes of the wavefront wrote (release, wave barrier, acquire).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace
}  // namespace plk
