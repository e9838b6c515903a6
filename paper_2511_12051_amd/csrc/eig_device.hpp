// Device building blocks of the per-pixel eigen-solve shared by the phase
// linking kernel and its adjoint: group reductions, FP64 and complex FP32
// Gauss-Jordan inversion with one LDS round trip per step, and shifted
// inverse iteration for the smallest eigenpair of a Hermitian matrix.
//
// A group of NP lanes (16 or 32, inside one wavefront) owns one pixel; lane i
// holds row i, NJ >= N columns.  LDS operations of one wavefront execute in
// program order, so exchanges within a group need no barrier.
#pragma once
#include <cmath>

#include "internal.hpp"

namespace plk {
namespace {

constexpr double kTauPivot = 1e-6;
constexpr float kTol2 = 4e-12f;  // squared change of the unit iterate at convergence
constexpr int kMaxIter = 96;
constexpr float kRefineRate = 0.5f;           // refine the shift when |dx| shrinks slower
__constant__ float kRefine[3] = {1.f, 2.f, 4.f};  // margins of the refined shifts, in residuals
constexpr int kBlock = 256;

__device__ __forceinline__ int lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0));
}

// Reductions over the NP lanes of a group.  Within a row of 16 lanes they use
// DPP lane permutations (quad swaps, half-row and row mirrors), so no LDS
// round trip is needed; a 32-lane group adds one exchange between rows.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}

template <int NP>
__device__ __forceinline__ float gsum(float v) {
    v += dpp<0xb1>(v);   // quad_perm [1,0,3,2]
    v += dpp<0x4e>(v);   // quad_perm [2,3,0,1]
    v += dpp<0x141>(v);  // row_half_mirror
    v += dpp<0x140>(v);  // row_mirror
#pragma unroll
    for (int o = 16; o < NP; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int NP>
__device__ __forceinline__ float gmax(float v) {
    v = fmaxf(v, dpp<0xb1>(v));
    v = fmaxf(v, dpp<0x4e>(v));
    v = fmaxf(v, dpp<0x141>(v));
    v = fmaxf(v, dpp<0x140>(v));
#pragma unroll
    for (int o = 16; o < NP; o <<= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

template <int NP>
__device__ __forceinline__ bool gany(bool p, int grp) {
    const uint64_t b = __ballot(p);
    const uint64_t m = (NP == 64 ? ~0ull : ((1ull << NP) - 1)) << (grp * NP);
    return (b & m) != 0;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// FP64 counterpart of publish_c without a shift.
template <int NJ>
__device__ __forceinline__ void publish_d(double (&g)[NJ], int k, double* buf) {
    const double p = g[k];
    const double inv = 1.0 / p;
#pragma unroll
    for (int j = 0; j < NJ; ++j) g[j] *= inv;
    g[k] = inv;
#pragma unroll
    for (int j = 0; j < NJ; ++j) buf[j] = g[j];
    buf[NJ] = p;
}

// Scales this lane's row k by 1/p, p = m[k] - mu, stores 1/p at k (in-place
// Gauss-Jordan form) and publishes the row and p for the group.
template <int NJ>
__device__ __forceinline__ void publish_c(float2 (&m)[NJ], int k, float mu, float2* buf) {
    const float p = m[k].x - mu;
    const float inv = 1.0f / p;
#pragma unroll
    for (int j = 0; j < NJ; ++j) m[j] = make_float2(m[j].x * inv, m[j].y * inv);
    m[k] = make_float2(inv, 0.f);
#pragma unroll
    for (int j = 0; j < NJ; ++j) buf[j] = m[j];
    buf[NJ] = make_float2(p, 0.f);
}

// In-place complex Gauss-Jordan inversion of the Hermitian matrix (m - mu I),
// row i of m being this lane's m[].  Lanes with act == false keep m unchanged.
// Returns (per group) whether every pivot was positive and finite.
// The shift is subtracted from each diagonal entry when its row becomes the
// pivot: earlier steps only add multiples of pivot rows to it, so this equals
// shifting first.  The lane owning row k+1 scales and publishes it right after
// its step-k update (double-buffered), so each step costs one LDS round trip.
// All lanes of a group belong to one wavefront and its LDS operations execute
// in program order, so no barrier is needed between publishing and reading.
template <int NJ>
__device__ __forceinline__ bool invert_c(float2 (&m)[NJ], float mu, int N, int i, bool act, float2* rb0, float2* rb1) {
    bool pd = true;
    if (act && i == 0) publish_c<NJ>(m, 0, mu, rb0);
#pragma unroll NJ
    for (int k = 0; k < NJ; ++k) {
        if (k < N) {
            const float2* buf = (k & 1) ? rb1 : rb0;
            float2* nbuf = (k & 1) ? rb0 : rb1;
            if (act) {
                const float p = buf[NJ].x;
                pd = pd && (p > 0.f) && (p <= 3.4e38f);
                if (i != k) {
                    const float2 f = m[k];
                    m[k] = make_float2(0.f, 0.f);
#pragma unroll
                    for (int j = 0; j < NJ; ++j) {
                        const float2 r = buf[j];
                        m[j].x = fmaf(-f.x, r.x, fmaf(f.y, r.y, m[j].x));
                        m[j].y = fmaf(-f.x, r.y, fmaf(-f.y, r.x, m[j].y));
                    }
                }
                if (k + 1 < N && i == k + 1) publish_c<NJ>(m, (k + 1 < NJ ? k + 1 : NJ - 1), mu, nbuf);
            }
        }
    }
    return pd;
}

template <int NJ>
__device__ __forceinline__ float2 matvec(const float2 (&m)[NJ], float2 x, int i, float2* xb) {
    xb[i] = x;  // read back below by the other lanes (in-order LDS)
    float2 y = make_float2(0.f, 0.f);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const float2 v = xb[j];
        y.x = fmaf(m[j].x, v.x, fmaf(-m[j].y, v.y, y.x));
        y.y = fmaf(m[j].x, v.y, fmaf(m[j].y, v.x, y.y));
    }
    return y;
}

// y_i = sum_j B_ij x_j with this lane's row of B in LDS (stride kBlock).
template <int NJ>
__device__ __forceinline__ float2 matvec_lds(const float2* brow, float2 x, int i, float2* xb) {
    xb[i] = x;
    float2 y = make_float2(0.f, 0.f);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const float2 v = xb[j], m = brow[j * kBlock];
        y.x = fmaf(m.x, v.x, fmaf(-m.y, v.y, y.x));
        y.y = fmaf(m.x, v.y, fmaf(m.y, v.x, y.y));
    }
    return y;
}

// In-place FP64 Gauss-Jordan inversion of G (row i = this lane's g[]) for
// lanes with act; returns (per group) whether some pivot was <= 1e-6 or not
// finite, i.e. the inversion failed.  Same publishing scheme as invert_c.
template <int NJ>
__device__ __forceinline__ bool invert_g(double (&g)[NJ], int N, int i, bool act, double* rbd0, double* rbd1) {
    bool fail = false;
    if (!gany<64>(act, 0)) return false;
    if (act && i == 0) publish_d<NJ>(g, 0, rbd0);
#pragma unroll NJ
    for (int k = 0; k < NJ; ++k) {
        if (k < N) {
            const double* buf = (k & 1) ? rbd1 : rbd0;
            double* nbuf = (k & 1) ? rbd0 : rbd1;
            if (act) {
                const double p = buf[NJ];
                fail = fail || !(p > kTauPivot && p <= 1.7976931348623157e308);
                if (i != k) {
                    const double f = g[k];
                    g[k] = 0.0;
#pragma unroll
                    for (int j = 0; j < NJ; ++j) g[j] = fma(-f, buf[j], g[j]);
                }
                if (k + 1 < N && i == k + 1) publish_d<NJ>(g, (k + 1 < NJ ? k + 1 : NJ - 1), nbuf);
            }
        }
    }
    return fail;
}

// Eigenvector of the smallest eigenvalue of the Hermitian B (this lane's
// row in LDS at bme[j * kBlock]) by shifted inverse iteration starting from
// x (unit norm, component ref_lane real and positive).  On return m holds
// (B - mu I)^{-1} for the last accepted shift, x the unit eigenvector
// component of this lane.
//
// Every iterate is rotated so that its component at ref_lane (the lane of the
// reference image in this group) is real and positive.  In FP32 the computed
// inverse is not exactly Hermitian, so its dominant eigenvalue carries a small
// phase; without the rotation each step turns the converged vector by that
// phase and the step length never falls below the tolerance.
template <int NP, int NJ>
__device__ __forceinline__ void eig_min(float2 (&m)[NJ], const float2* bme, float bnorm2, float mu, bool solve,
                        int N, int i, int ref_lane, float2* rbc0, float2* rbc1, float2* xb, float2& x,
                        bool& conv, int& it, int& retries) {
    // One factorisation site serves the first shift and its back-off
    // schedule, the refined shifts, and restoring the accepted shift after
    // every refined candidate was rejected.
#pragma unroll NJ
    for (int j = 0; j < NJ; ++j) m[j] = make_float2(0.f, 0.f);
    float mu_req = mu;    // shift of the pending factorisation
    bool need = solve;    // this group waits for a factorisation
    int stage = 0;        // 0..3: first-shift schedule, 4: refining, 5: restoring
    int cand = 0;         // refined candidate rho - kRefine[cand] * res
    float rho_t = 0.f, res_t = 0.f;
    conv = !solve;
    it = 0;
    retries = 0;
    float d2prev = 0.f;
    for (int guard = 0; guard < 2 * kMaxIter; ++guard) {
        if (gany<64>(need, 0)) {
#pragma unroll NJ
            for (int j = 0; j < NJ; ++j) if (need) m[j] = bme[j * kBlock];
            const bool ok = invert_c<NJ>(m, mu_req, N, i, need, rbc0, rbc1);
            if (need) {
                if (ok) {
                    if (stage == 4) d2prev = 0.f;  // the contraction rate changes
                    mu = mu_req;
                    need = false;
                    stage = stage < 4 ? stage : 4;
                } else if (stage == 4) {
                    ++retries;
                    ++cand;
                    const float next = cand < 3 ? rho_t - kRefine[cand] * res_t : mu;
                    if (next > mu) {
                        mu_req = next;
                    } else {  // every candidate rejected: factor the accepted shift again
                        mu_req = mu;
                        stage = 5;
                    }
                } else if (stage == 5) {  // cannot happen in exact arithmetic
                    need = false;
                    conv = true;
                } else {  // first shift rejected: back off
                    ++retries;
                    ++stage;
                    if (stage == 1) mu_req = 0.5f;
                    else if (stage == 2) mu_req = 0.0f;
                    else if (stage == 3) {
                        mu_req = -sqrtf(gsum<NP>(bnorm2)) - 1.0f;  // below -||B||_F <= lambda_min
                    } else {
                        need = false;
                        conv = true;
                    }
                }
            }
            continue;
        }
        if (!gany<64>(!conv, 0) || it >= kMaxIter) break;
        float2 y = matvec<NJ>(m, x, i, xb);
        const float n2 = gsum<NP>(y.x * y.x + y.y * y.y);
        const float2 yr = make_float2(__shfl(y.x, ref_lane, 64), __shfl(y.y, ref_lane, 64));
        const float r2 = yr.x * yr.x + yr.y * yr.y;
        // scale by conj(y_ref) / (|y_ref| ||y||); plain 1/||y|| if y_ref vanishes
        const bool gauge = r2 > 1e-30f * n2;
        const float sc = gauge ? 1.0f / sqrtf(n2 * r2) : 1.0f / sqrtf(n2);
        const float2 u = gauge ? make_float2(yr.x * sc, -yr.y * sc) : make_float2(sc, 0.f);
        y = cmul(y, u);
        const float dx = y.x - x.x, dy = y.y - x.y;
        const float d2 = gsum<NP>(dx * dx + dy * dy);
        const bool finite = n2 > 0.f && n2 <= 3.4e38f;
        // contraction rate of the iteration (1 until two steps are known)
        const float q2 = d2prev > 0.f ? d2 / d2prev : 1.f;
        if (!conv) {
            if (finite) x = y;
            if (d2 < kTol2 || !finite) conv = true;
            d2prev = d2;
        }
        ++it;
        if (it == 4 || it == 8 || it == 12 || it == 18) {
            // slow contraction: move the shift towards lambda_min.  The first
            // candidate rho - ||Bx - rho x|| bounds the eigenvalue nearest rho
            // from below; while x still mixes several eigenvectors it can lie
            // above lambda_min, so larger margins follow if the inertia check
            // rejects it.
            const bool slow = !conv && q2 > kRefineRate * kRefineRate;
            if (gany<64>(slow, 0)) {
                const float2 bx = matvec_lds<NJ>(bme, x, i, xb);
                const float rho = gsum<NP>(x.x * bx.x + x.y * bx.y);
                const float rx = bx.x - rho * x.x, ry = bx.y - rho * x.y;
                const float res = sqrtf(gsum<NP>(rx * rx + ry * ry));
                if (slow && rho - res > mu) {
                    rho_t = rho;
                    res_t = res;
                    cand = 0;
                    mu_req = rho - res;
                    need = true;
                    stage = 4;
                }
            }
        }
    }

}

}  // namespace
}  // namespace plk
