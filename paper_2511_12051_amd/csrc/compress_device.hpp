// Device body of the compressed SLC: one thread (tid of a kBlock-thread
// block) per full-resolution pixel.  See compress.hip.
#pragma once
#include "internal.hpp"
#include "lanes.hpp"

namespace plk {
namespace {

typedef float f32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void compress_body(const CompressArgs& a, int64_t block_x, int64_t y, int tid) {
    const PlaneTable& t = a.t;
    const Geometry& g = a.g;
    const int N = a.N, first_real = a.first_real;
    const float2* __restrict__ ph = a.ph;
    float2* __restrict__ kappa = a.kappa;
    const int64_t x = block_x * kBlock + tid;
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
    if (a.rot >= 0) {  // times phasor rot: the sum re-referenced to image rot
        const float2 w = ph[(int64_t)a.rot * opix + b];
        const float r2 = re * w.x - im * w.y;
        im = re * w.y + im * w.x;
        re = r2;
    }
    kappa[p] = make_float2(re, im);
}

// compress_body over the blocks b, b + 2, b + 4, b + 6 below `end` at once,
// each plane's four loads issued together.  The same arithmetic per pixel.
__device__ __forceinline__ void compress_body4(const CompressArgs& a, int64_t b, int64_t end, int tid) {
    const PlaneTable& t = a.t;
    const Geometry& g = a.g;
    const int N = a.N, first_real = a.first_real;
    const int64_t opix = g.oR * g.oC;
    int64_t p[4], blk[4];
    bool on[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t bq = b + 2 * q;
        const int64_t bx = bq % a.gx, y = bq / a.gx;
        const int64_t x = bx * kBlock + tid;
        on[q] = bq < end && x < g.C;
        int64_t oy = y / g.sy, ox = x / g.sx;
        oy = oy < g.oR - 1 ? oy : g.oR - 1;
        ox = ox < g.oC - 1 ? ox : g.oC - 1;
        blk[q] = on[q] ? oy * g.oC + ox : 0;
        p[q] = on[q] ? y * g.C + x : 0;
    }
    float re[4] = {0.f, 0.f, 0.f, 0.f}, im[4] = {0.f, 0.f, 0.f, 0.f};
    for (int i = first_real; i < N; ++i) {
        f32x2 z[4];
        float2 w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            z[q] = __builtin_nontemporal_load(reinterpret_cast<const f32x2*>(t.p[i]) + p[q]);
            w[q] = a.ph[(int64_t)i * opix + blk[q]];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            re[q] = fmaf(w[q].x, z[q].x, fmaf(w[q].y, z[q].y, re[q]));
            im[q] = fmaf(w[q].x, z[q].y, fmaf(-w[q].y, z[q].x, im[q]));
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        float r = re[q], m = im[q];
        if (a.rot >= 0) {
            const float2 w = a.ph[(int64_t)a.rot * opix + blk[q]];
            const float r2 = r * w.x - m * w.y;
            m = r * w.y + m * w.x;
            r = r2;
        }
        if (on[q]) a.kappa[p[q]] = make_float2(r, m);
    }
}

}  // namespace
}  // namespace plk
