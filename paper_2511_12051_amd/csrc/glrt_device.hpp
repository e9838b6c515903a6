// Device body of the GLRT selection: one workgroup per tile of TX x TY
// output pixels (any block size of at least TX * TY threads).  See glrt.hip.
#pragma once
#include <cmath>

#include "internal.hpp"

namespace plk {
namespace {

constexpr double kRecheckRel = 1e-8;
constexpr double kBand = 1e-9;

// tid / nthreads: this thread and the threads (at least TX * TY) that work
// on the tile; every thread of the workgroup reaches the one barrier.
__device__ __forceinline__ void glrt_body(const GlrtArgs& a, int64_t bx, int64_t by, double* s_tile, int tid,
                                          int nthreads) {
    const Geometry& g = a.g;
    const int64_t oy0 = by * a.TY, ox0 = bx * a.TX;
    const int64_t y0 = oy0 * g.sy + g.sy / 2 - g.hy;
    const int64_t x0 = ox0 * g.sx + g.sx / 2 - g.hx;
    const int nt = a.tw * a.th;
    // The tile is staged kU elements per thread at a time: their loads are
    // issued together (at clamped in-image indices, so without branches)
    // before any is used, instead of one load pair and one wait per element.
    constexpr int kU = 8;
    for (int i0 = tid; i0 < nt; i0 += kU * nthreads) {
        double m[kU], v[kU];
        bool in[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int i = i0 + u * nthreads;
            const int ly = i / a.tw, lx = i - ly * a.tw;
            const int64_t y = y0 + ly, x = x0 + lx;
            in[u] = i < nt && y >= 0 && y < g.R && x >= 0 && x < g.C;
            const int64_t p = in[u] ? y * g.C + x : 0;
            m[u] = a.mean[p];
            v[u] = a.var[p];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int i = i0 + u * nthreads;
            double s = __builtin_nan("");
            if (in[u]) {
                const double sv = 0.5 * fma(m[u], m[u], v[u]);
                if (sv > 0.0 && sv <= 1.7976931348623157e308) s = sv;
            }
            if (i < nt) s_tile[i] = s;
        }
    }
    __syncthreads();

    const int ly = tid / a.TX, lx = tid - ly * a.TX;
    const int64_t oy = oy0 + ly, ox = ox0 + lx;
    if (ly >= a.TY || oy >= g.oR || ox >= g.oC) return;
    const double* row0 = s_tile + (ly * g.sy) * a.tw + lx * g.sx;
    const double sp = row0[g.hy * a.tw + g.hx];
    const bool pvalid = sp == sp;
    const double lo = a.rlo * sp, hi = a.rhi * sp;
    const double lo_tol = kRecheckRel * lo, hi_tol = kRecheckRel * hi;
    const int64_t pix = oy * g.oC + ox;
    uint32_t* out = a.mask + pix * g.nw;
    uint32_t word = 0;
    int bit = 0, wi = 0, cnt = 0;
    unsigned long long band = 0, rechecks = 0;
    for (int dy = 0; dy < g.wy; ++dy) {
        const double* row = row0 + dy * a.tw;
        for (int dx = 0; dx < g.wx; ++dx) {
            const double sq = row[dx];
            bool ok;
            if (dy == g.hy && dx == g.hx) {
                ok = true;
            } else if (!pvalid) {
                ok = false;
            } else {
                ok = (sq >= lo) && (sq <= hi);  // false for NaN
                if (fabs(sq - hi) <= hi_tol || fabs(sq - lo) <= lo_tol) {
                    const double t = 2.0 * a.n * (2.0 * log((sp + sq) * 0.5) - log(sp) - log(sq));
                    ok = t <= a.thr;
                    ++rechecks;
                    if (fabs(t - a.thr) < kBand) ++band;
                }
            }
            word |= (uint32_t)ok << bit;
            cnt += ok;
            if (++bit == 32) {
                out[wi++] = word;
                word = 0;
                bit = 0;
            }
        }
    }
    if (bit) out[wi] = word;
    a.count[pix] = (uint16_t)cnt;
    if (a.counters && (band | rechecks)) {
        atomicAdd(a.counters + PL_CNT_GLRT_BAND, band);
        atomicAdd(a.counters + PL_CNT_GLRT_RECHECK, rechecks);
    }
}

}  // namespace
}  // namespace plk
