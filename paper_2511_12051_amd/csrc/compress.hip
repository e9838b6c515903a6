// Compressed SLC of a mini-stack (paper Sec. 2.2): kappa = zeta^H z over the
// real images, each full-resolution pixel using the linked phasors of its
// decimation block.  HBM-bound: one thread per pixel, coalesced plane reads;
// the phasor reads hit in cache (one block serves stride_x * stride_y pixels).
#include "internal.hpp"

namespace plk {
namespace {

constexpr int kBlock = 256;
typedef float f32x2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(kBlock) void compress_kernel(PlaneTable t, int N, int first_real,
                                                          Geometry g, const float2* __restrict__ ph,
                                                          float2* __restrict__ kappa) {
    const int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t y = blockIdx.y;
    if (x >= g.C) return;
    int64_t by = y / g.sy, bx = x / g.sx;
    by = by < g.oR - 1 ? by : g.oR - 1;
    bx = bx < g.oC - 1 ? bx : g.oC - 1;
    const int64_t opix = g.oR * g.oC;
    const int64_t b = by * g.oC + bx;
    const int64_t p = y * g.C + x;
    float re = 0.f, im = 0.f;
    for (int i = first_real; i < N; ++i) {
        const f32x2 z = __builtin_nontemporal_load(reinterpret_cast<const f32x2*>(t.p[i]) + p);
        float2 w = ph[(int64_t)i * opix + b];
        // conj(w) * z
        re = fmaf(w.x, z.x, fmaf(w.y, z.y, re));
        im = fmaf(w.x, z.y, fmaf(-w.y, z.x, im));
    }
    kappa[p] = make_float2(re, im);
}

}  // namespace

pl_status launch_compress(const PlaneTable& t, int N, int first_real, const Geometry& g,
                          const float2* phasors, float2* kappa, hipStream_t s) {
    if (g.R > 2147483647LL) return fail(PL_ERR_UNSUPPORTED, "pl_compress_ministack: too many rows");
    dim3 grid((unsigned)((g.C + kBlock - 1) / kBlock), (unsigned)g.R);
    hipLaunchKernelGGL(compress_kernel, grid, dim3(kBlock), 0, s, t, N, first_real, g, phasors, kappa);
    return launch_ok("compress kernel");
}

}  // namespace plk
