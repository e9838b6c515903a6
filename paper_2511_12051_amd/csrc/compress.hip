// Compressed SLC of a mini-stack (paper Sec. 2.2): kappa = zeta^H z over the
// real images, each full-resolution pixel using the linked phasors of its
// decimation block.  HBM-bound: one thread per pixel, coalesced plane reads;
// the phasor reads hit in cache (one block serves stride_x * stride_y pixels).
#include "batch_device.hpp"
#include "compress_device.hpp"
#include "internal.hpp"

namespace plk {
namespace {

__global__ __launch_bounds__(kBlock) void compress_kernel(CompressArgs a) { compress_body(a, blockIdx.x, blockIdx.y, threadIdx.x); }

__global__ __launch_bounds__(kBlock) void compress_batch(BatchRange<CompressArgs> r) {
    for (int64_t b = blockIdx.x; b < r.total; b += gridDim.x) {
        const int k = batch_item(r.starts, r.n, b);
        const CompressArgs& a = r.items[k];
        const int64_t local = b - r.starts[k];
        compress_body(a, local % a.gx, local / a.gx, threadIdx.x);
    }
}

}  // namespace

CompressArgs compress_args(const PlaneTable& t, int N, int first_real, const Geometry& g,
                           const float2* phasors, float2* kappa, int64_t* blocks) {
    CompressArgs a{t, N, first_real, g, phasors, kappa, (g.C + kBlock - 1) / kBlock, -1};
    *blocks = a.gx * g.R;
    return a;
}

pl_status launch_compress(const PlaneTable& t, int N, int first_real, const Geometry& g,
                          const float2* phasors, float2* kappa, hipStream_t s, int rot) {
    if (g.R > 2147483647LL) return fail(PL_ERR_UNSUPPORTED, "pl_compress_ministack: too many rows");
    int64_t blocks;
    CompressArgs a = compress_args(t, N, first_real, g, phasors, kappa, &blocks);
    a.rot = rot;
    dim3 grid((unsigned)a.gx, (unsigned)g.R);
    hipLaunchKernelGGL(compress_kernel, grid, dim3(kBlock), 0, s, a);
    return launch_ok("compress kernel");
}

const void* compress_batch_fn() { return reinterpret_cast<const void*>(compress_batch); }

pl_status launch_compress_batch(const BatchRange<CompressArgs>& r, int64_t grid, hipStream_t s) {
    if (r.total == 0) return PL_OK;
    hipLaunchKernelGGL(compress_batch, dim3((unsigned)grid), dim3(kBlock), 0, s, r);
    return launch_ok("batched compress kernel");
}

}  // namespace plk
