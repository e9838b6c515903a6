// Amplitude statistics and their pooled merge (paper Sec. 3.1,
// eq. merged-mean and eq. merged-variance).  HBM-bound streaming kernels:
// one thread per two adjacent pixels, 16-byte loads, FP64 accumulation.
#include "batch_device.hpp"
#include "internal.hpp"
#include "stats_device.hpp"

namespace plk {
namespace {

__global__ __launch_bounds__(kBlock) void amp_stats_vec(StatsArgs a) { stats_vec_body(a, blockIdx.x, threadIdx.x); }
__global__ __launch_bounds__(kBlock) void amp_stats_scalar(StatsArgs a) { stats_scalar_body(a, blockIdx.x, threadIdx.x); }

template <bool VEC>
__global__ __launch_bounds__(kBlock) void amp_stats_batch(BatchRange<StatsArgs> r) {
    for (int64_t b = blockIdx.x; b < r.total; b += gridDim.x) {
        const int k = batch_item(r.starts, r.n, b);
        if (VEC) stats_vec_body(r.items[k], b - r.starts[k], threadIdx.x);
        else stats_scalar_body(r.items[k], b - r.starts[k], threadIdx.x);
    }
}

struct GroupTable {
    const double* mean[64];
    const double* var[64];
    double w[64];
};

__global__ __launch_bounds__(kBlock) void merge_stats_kernel(GroupTable g, int G, double wsum_inv,
                                                             int64_t npix, double* mean_out,
                                                             double* var_out) {
    int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= npix) return;
    double mu = 0.0, second = 0.0;
    for (int i = 0; i < G; ++i) {
        double m = g.mean[i][p], v = g.var[i][p];
        mu = fma(g.w[i], m, mu);
        second = fma(g.w[i], fma(m, m, v), second);
    }
    mu *= wsum_inv;
    second *= wsum_inv;
    mean_out[p] = mu;
    var_out[p] = second - mu * mu;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

}  // namespace

bool stats_args(const PlaneTable& t, int first, int M, int64_t npix, double* mean, double* var,
                StatsArgs* a, int64_t* blocks) {
    bool vec = (npix % 2 == 0) && aligned16(mean) && aligned16(var);
    for (int m = 0; m < M && vec; ++m) vec = aligned16(t.p[first + m]);
    *a = StatsArgs{t, first, M, vec ? npix / 2 : npix, mean, var};
    *blocks = (a->n + kBlock - 1) / kBlock;
    return vec;
}

pl_status launch_amp_stats(const PlaneTable& t, int first, int M, int64_t npix, double* mean,
                           double* var, hipStream_t s) {
    StatsArgs a;
    int64_t blocks;
    const bool vec = stats_args(t, first, M, npix, mean, var, &a, &blocks);
    if (vec) hipLaunchKernelGGL(amp_stats_vec, dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL(amp_stats_scalar, dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
    return launch_ok("amplitude statistics kernel");
}

const void* amp_stats_batch_fn(bool vec) {
    return vec ? reinterpret_cast<const void*>(amp_stats_batch<true>) : reinterpret_cast<const void*>(amp_stats_batch<false>);
}

pl_status launch_amp_stats_batch(const BatchRange<StatsArgs>& r, bool vec, int64_t grid, hipStream_t s) {
    if (r.total == 0) return PL_OK;
    if (vec) hipLaunchKernelGGL(amp_stats_batch<true>, dim3((unsigned)grid), dim3(kBlock), 0, s, r);
    else hipLaunchKernelGGL(amp_stats_batch<false>, dim3((unsigned)grid), dim3(kBlock), 0, s, r);
    return launch_ok("batched amplitude statistics kernel");
}

pl_status launch_merge_stats(const double* const* means, const double* const* vars,
                             const double* weights, int G, int64_t npix, double* mean_out,
                             double* var_out, hipStream_t s) {
    GroupTable g{};
    double wsum = 0.0;
    for (int i = 0; i < G; ++i) {
        g.mean[i] = means[i];
        g.var[i] = vars[i];
        g.w[i] = weights[i];
        wsum += weights[i];
    }
    int64_t blocks = (npix + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(merge_stats_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, g, G,
                       1.0 / wsum, npix, mean_out, var_out);
    return launch_ok("statistics merge kernel");
}

}  // namespace plk
