// GLRT selection of statistically homogeneous pixels (paper Sec. 3.1).
//
// A workgroup owns a tile of TX x TY output pixels and stages the Rayleigh
// scale s = (mean^2 + var)/2 of the input pixels its windows cover in LDS
// (FP64; NaN outside the image or where s is not finite and positive).  One
// thread per output pixel walks its window in the mask's bit order.
//
// With n samples, T = 2n ln((s_p+s_q)^2 / (4 s_p s_q)) <= thr holds exactly
// when r = s_q/s_p lies in [1/r_hi, r_hi], r_hi = 2c-1 + 2 sqrt(c^2-c),
// c = exp(thr/2n), so almost every pair costs two FP64 multiplies and
// compares.  Pairs whose scale lies within 1e-8 (relative) of either bound
// are re-decided with the logarithmic form itself, and those with
// |T - thr| < 1e-9 are counted.
#include <cmath>

#include "batch_device.hpp"
#include "glrt_device.hpp"
#include "internal.hpp"

namespace plk {
namespace {

// chi-square (1 dof) upper quantile: thr = z^2 with erfc(z / sqrt(2)) = alpha,
// found by bisection on the monotone erfc in long double.
double chi2_1_isf(double alpha) {
    long double lo = 0.0L, hi = 40.0L;
    for (int i = 0; i < 200; ++i) {  // bisection to full precision
        long double mid = 0.5L * (lo + hi);
        if (erfcl(mid / sqrtl(2.0L)) > (long double)alpha) lo = mid; else hi = mid;
    }
    long double z = 0.5L * (lo + hi);
    return (double)(z * z);
}

__global__ __launch_bounds__(256) void glrt_kernel(GlrtArgs a) {
    extern __shared__ double s_tile[];
    glrt_body(a, blockIdx.x, blockIdx.y, s_tile, threadIdx.x, blockDim.x);
}

__global__ __launch_bounds__(256) void glrt_batch(BatchRange<GlrtArgs> r) {
    extern __shared__ double s_tile[];
    for (int64_t b = blockIdx.x; b < r.total; b += gridDim.x) {
        const int k = batch_item(r.starts, r.n, b);
        const GlrtArgs& a = r.items[k];
        const int64_t local = b - r.starts[k];
        glrt_body(a, local % a.gx, local / a.gx, s_tile, threadIdx.x, blockDim.x);
        __syncthreads();  // the tile is refilled by the next block
    }
}

}  // namespace

bool glrt_args(const double* mean, const double* var, const Geometry& g, double n_eff, double alpha,
               uint32_t* mask, uint16_t* count, unsigned long long* counters, GlrtArgs* out,
               int64_t* blocks, size_t* lds) {
    GlrtArgs a{};
    a.mean = mean;
    a.var = var;
    a.g = g;
    a.mask = mask;
    a.count = count;
    a.counters = counters;
    a.n = n_eff;
    a.thr = chi2_1_isf(alpha);
    long double c = expl((long double)a.thr / (2.0L * (long double)n_eff));
    long double rhi = 2.0L * c - 1.0L + 2.0L * sqrtl(c * c - c);
    a.rhi = (double)rhi;
    a.rlo = (double)(1.0L / rhi);
    const size_t budget = 64 * 1024;
    static const int shapes[][2] = {{16, 16}, {32, 8}, {16, 8}, {8, 8}, {8, 4}, {4, 4}, {4, 2}, {2, 2}, {1, 1}};
    for (auto& sh : shapes) {
        a.TX = sh[0];
        a.TY = sh[1];
        a.tw = (a.TX - 1) * g.sx + g.wx;
        a.th = (a.TY - 1) * g.sy + g.wy;
        if ((size_t)a.tw * a.th * sizeof(double) <= budget) break;
    }
    *lds = (size_t)a.tw * a.th * sizeof(double);
    a.gx = (g.oC + a.TX - 1) / a.TX;
    *blocks = a.gx * ((g.oR + a.TY - 1) / a.TY);
    *out = a;
    return *lds <= budget;
}

pl_status launch_shp_select(const double* mean, const double* var, const Geometry& g,
                            double n_eff, double alpha, uint32_t* mask, uint16_t* count,
                            unsigned long long* counters, hipStream_t s) {
    GlrtArgs a;
    int64_t blocks;
    size_t lds;
    if (!glrt_args(mean, var, g, n_eff, alpha, mask, count, counters, &a, &blocks, &lds))
        return fail(PL_ERR_UNSUPPORTED, "pl_shp_select: window/stride too large for LDS");
    dim3 grid((unsigned)a.gx, (unsigned)((g.oR + a.TY - 1) / a.TY));
    if (grid.y > 65535) return fail(PL_ERR_UNSUPPORTED, "pl_shp_select: output grid too tall");
    hipLaunchKernelGGL(glrt_kernel, grid, dim3(a.TX * a.TY), lds, s, a);
    return launch_ok("GLRT kernel");
}

const void* glrt_batch_fn() { return reinterpret_cast<const void*>(glrt_batch); }

pl_status launch_shp_select_batch(const BatchRange<GlrtArgs>& r, int threads, size_t lds, int64_t grid,
                                  hipStream_t s) {
    if (r.total == 0) return PL_OK;
    hipLaunchKernelGGL(glrt_batch, dim3((unsigned)grid), dim3(threads), lds, s, r);
    return launch_ok("batched GLRT kernel");
}

}  // namespace plk
