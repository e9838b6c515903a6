// Device bodies of the amplitude statistics (per pixel pair and per pixel);
// block of kBlock threads, tid its thread.  See stats.hip.
#pragma once
#include <cmath>

#include "internal.hpp"
#include "lanes.hpp"

namespace plk {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Shifted single-pass moments: with K the first amplitude of the pixel,
// s = sum(a - K), q = sum((a - K)^2) give mean = K + s/M and the population
// variance (q - s^2/M)/M without the cancellation of sum(a^2) - M mean^2.
struct Moments {
    double k = 0, s = 0, q = 0;
    __device__ void add(double a, int m) {
        if (m == 0) k = a;
        double d = a - k;
        s += d;
        q = fma(d, d, q);
    }
    __device__ void finish(int M, double* mean, double* var) const {
        double inv = 1.0 / (double)M;
        *mean = k + s * inv;
        double v = (q - s * s * inv) * inv;
        *var = v > 0.0 ? v : 0.0;
    }
};

__device__ inline double amp(float re, float im) {
    double r = re, i = im;
    return sqrt(fma(r, r, i * i));
}

// 16-byte aligned planes with an even pixel count: one float4 = two pixels.
__device__ __forceinline__ void stats_vec_body(const StatsArgs& a, int64_t block, int tid) {
    int64_t j = block * kBlock + tid;
    if (j >= a.n) return;
    Moments u, w;
    for (int m = 0; m < a.M; ++m) {
        const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(a.t.p[a.first + m]) + j);
        u.add(amp(v.x, v.y), m);
        w.add(amp(v.z, v.w), m);
    }
    double m0, v0, m1, v1;
    u.finish(a.M, &m0, &v0);
    w.finish(a.M, &m1, &v1);
    reinterpret_cast<double2*>(a.mean)[j] = make_double2(m0, m1);
    reinterpret_cast<double2*>(a.var)[j] = make_double2(v0, v1);
}

__device__ __forceinline__ void stats_scalar_body(const StatsArgs& a, int64_t block, int tid) {
    int64_t p = block * kBlock + tid;
    if (p >= a.n) return;
    Moments u;
    for (int m = 0; m < a.M; ++m) {
        float2 v = a.t.p[a.first + m][p];
        u.add(amp(v.x, v.y), m);
    }
    u.finish(a.M, a.mean + p, a.var + p);
}

}  // namespace
}  // namespace plk
