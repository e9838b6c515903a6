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
// round trip is needed; wider groups add exchanges between rows.
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

// |z| of an FP32 complex value to about 1e-14 relative, without the FP64
// square-root sequence: exact sum of squares in FP64, an FP32 reciprocal
// square root as seed and one Newton step in FP64 (the seed's 2^-23 relative
// error becomes ~1e-14).
__device__ __forceinline__ double cabs64(float re, float im) {
    const double x = fma((double)re, (double)re, (double)im * (double)im);
    if (!(x > 1e-30) || x > 1e30) return sqrt(x);  // tiny, huge or not finite: the exact path
    double y = (double)__builtin_amdgcn_rsqf((float)x);
    y = y * fma(-0.5 * x * y, y, 1.5);
    return x * y;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Gauss-Jordan with deferred row scaling.  Lane i stores its row unscaled,
// S_i, with a scale sig_i: the true row is sig_i S_i.  At step k the pivot
// lane publishes S_k with its diagonal slot set to 1, the pivot p and
// sig_k = 1/p, and keeps them; every other lane i updates
//   S_i[j] -= (S_i[k] sig_k) S_k[j]  (after setting S_i[k] = 0),
// which is the in-place Gauss-Jordan step divided through by sig_i.  Nobody
// rescales a row during the sweep (the pivot lane alone used to, with the
// rest of the wavefront idle); each lane scales its row once at the end.

// FP64 pivot row: p = g[k] (no shift); sig = 1/p by a hardware reciprocal
// refined twice by Newton's method.
template <int NJ>
__device__ __forceinline__ void publish_d(double (&g)[NJ], int k, double* buf, double& sig) {
    const double p = g[k];
    double r = __builtin_amdgcn_rcp(p);
    r = fma(r, fma(-p, r, 1.0), r);
    r = fma(r, fma(-p, r, 1.0), r);
    sig = r;
    g[k] = 1.0;
#pragma unroll
    for (int j = 0; j < NJ; ++j) buf[j] = g[j];
    buf[NJ] = p;
    buf[NJ + 1] = r;
}

// Complex pivot row of (m - mu I): p = m[k] - mu (the shift is applied when a
// row becomes the pivot; earlier steps only add multiples of pivot rows to
// it, so this equals shifting first).
template <int NJ>
__device__ __forceinline__ void publish_c(float2 (&m)[NJ], int k, float mu, float2* buf, float& sig) {
    const float p = m[k].x - mu;
    const float r = __builtin_amdgcn_rcpf(p);
    sig = r;
    m[k] = make_float2(1.f, 0.f);
#pragma unroll
    for (int j = 0; j < NJ; ++j) buf[j] = m[j];
    buf[NJ] = make_float2(p, r);
}

// In-place complex Gauss-Jordan inversion of the Hermitian matrix (m - mu I),
// row i of m being this lane's m[].  Lanes with act == false keep m unchanged.
// Returns (per group) whether every pivot was positive and finite, which by
// Sylvester's law of inertia proves mu below the smallest eigenvalue.
// The lane owning row k+1 publishes it right after its step-k update
// (double-buffered), so each step costs one LDS round trip.  All lanes of a
// group belong to one wavefront and its LDS operations execute in program
// order, so no barrier is needed between publishing and reading.
template <int NJ>
__device__ __forceinline__ bool invert_c(float2 (&m)[NJ], float mu, int N, int i, bool act, float2* rb0, float2* rb1) {
    bool pd = true;
    float sig = 1.f;
    if (act && i == 0) publish_c<NJ>(m, 0, mu, rb0, sig);
#pragma unroll NJ
    for (int k = 0; k < NJ; ++k) {
        if (k < N) {
            const float2* buf = (k & 1) ? rb1 : rb0;
            float2* nbuf = (k & 1) ? rb0 : rb1;
            if (act) {
                const float2 ps = buf[NJ];
                pd = pd && (ps.x > 0.f) && (ps.x <= 3.4e38f);
                if (i != k) {
                    const float2 f = make_float2(m[k].x * ps.y, m[k].y * ps.y);
                    m[k] = make_float2(0.f, 0.f);
#pragma unroll
                    for (int j = 0; j < NJ; ++j) {
                        const float2 r = buf[j];
                        m[j].x = fmaf(-f.x, r.x, fmaf(f.y, r.y, m[j].x));
                        m[j].y = fmaf(-f.x, r.y, fmaf(-f.y, r.x, m[j].y));
                    }
                }
                if (k + 1 < N && i == k + 1) publish_c<NJ>(m, (k + 1 < NJ ? k + 1 : NJ - 1), mu, nbuf, sig);
            }
        }
    }
    if (act) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) m[j] = make_float2(m[j].x * sig, m[j].y * sig);
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

// ---- 16-lane groups: exchanges by DPP row broadcast.  A group of 16 lanes
// is one DPP row, and row_newbcast:L hands lane L's register to every lane of
// the row inside the instruction's operand path.  The pivot row of a
// Gauss-Jordan step (held by the pivot lane) and the iterate of a mat-vec
// (one component per lane) then move between lanes without LDS traffic or
// its round-trip latency.  The arithmetic, and its order, is that of the LDS
// versions above, so both give identical results.
template <int L>
__device__ __forceinline__ float rowcast(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x150 + L, 0xf, 0xf, true));
}
template <int L>
__device__ __forceinline__ double rowcast(double v) {
    return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + L, 0xf, 0xf, true);
}

// Step K onwards of the complex Gauss-Jordan inversion of (m - mu I) with
// deferred row scaling: every lane reads the pivot p = m_K[K] - mu and forms
// sig = 1/p itself; the pivot lane keeps its row S_K with the diagonal slot
// set to 1, every other active lane i subtracts (S_i[K] sig) S_K.
template <int NJ, int K>
__device__ __forceinline__ void invert_c16_steps(float2 (&m)[NJ], float mu, int N, int i, bool act,
                                                 bool& pd, float& sig) {
    if constexpr (K < NJ) {
        if (K < N) {
            const float p = rowcast<K>(m[K].x) - mu;
            pd = pd && (p > 0.f) && (p <= 3.4e38f);
            const float r = __builtin_amdgcn_rcpf(p);
            const bool piv = i == K;
            sig = piv ? r : sig;
            const bool upd = act && !piv;
            const float fx = upd ? m[K].x * r : 0.f;
            const float fy = upd ? m[K].y * r : 0.f;
            if (act) m[K] = piv ? make_float2(1.f, 0.f) : make_float2(0.f, 0.f);
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const float rx = rowcast<K>(m[j].x), ry = rowcast<K>(m[j].y);
                m[j].x = fmaf(-fx, rx, fmaf(fy, ry, m[j].x));
                m[j].y = fmaf(-fx, ry, fmaf(-fy, rx, m[j].y));
            }
        }
        invert_c16_steps<NJ, K + 1>(m, mu, N, i, act, pd, sig);
    }
}

template <int NJ>
__device__ __forceinline__ bool invert_c16(float2 (&m)[NJ], float mu, int N, int i, bool act) {
    static_assert(NJ <= 16, "one row of 16 lanes per group");
    bool pd = true;
    float sig = 1.f;
    invert_c16_steps<NJ, 0>(m, mu, N, i, act, pd, sig);
    if (act) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) m[j] = make_float2(m[j].x * sig, m[j].y * sig);
    }
    return pd;
}

template <int NJ, int J>
__device__ __forceinline__ void matvec16_steps(const float2 (&m)[NJ], float2 x, float2& y) {
    if constexpr (J < NJ) {
        const float vx = rowcast<J>(x.x), vy = rowcast<J>(x.y);
        y.x = fmaf(m[J].x, vx, fmaf(-m[J].y, vy, y.x));
        y.y = fmaf(m[J].x, vy, fmaf(m[J].y, vx, y.y));
        matvec16_steps<NJ, J + 1>(m, x, y);
    }
}

template <int NJ, int J>
__device__ __forceinline__ void matvec16_lds_steps(const float2* brow, float2 x, float2& y) {
    if constexpr (J < NJ) {
        const float2 m = brow[J * kBlock];
        const float vx = rowcast<J>(x.x), vy = rowcast<J>(x.y);
        y.x = fmaf(m.x, vx, fmaf(-m.y, vy, y.x));
        y.y = fmaf(m.x, vy, fmaf(m.y, vx, y.y));
        matvec16_lds_steps<NJ, J + 1>(brow, x, y);
    }
}

template <int NJ, int K>
__device__ __forceinline__ void invert_g16_steps(double (&g)[NJ], int N, int i, bool act, bool& fail, double& sig) {
    if constexpr (K < NJ) {
        if (K < N) {
            const double p = rowcast<K>(g[K]);
            fail = fail || (act && !(p > kTauPivot && p <= 1.7976931348623157e308));
            double r = __builtin_amdgcn_rcp(p);
            r = fma(r, fma(-p, r, 1.0), r);
            r = fma(r, fma(-p, r, 1.0), r);
            const bool piv = i == K;
            sig = piv ? r : sig;
            const double f = (act && !piv) ? g[K] * r : 0.0;
            if (act) g[K] = piv ? 1.0 : 0.0;
#pragma unroll
            for (int j = 0; j < NJ; ++j) g[j] = fma(-f, rowcast<K>(g[j]), g[j]);
        }
        invert_g16_steps<NJ, K + 1>(g, N, i, act, fail, sig);
    }
}

template <int NJ>
__device__ __forceinline__ bool invert_g16(double (&g)[NJ], int N, int i, bool act) {
    static_assert(NJ <= 16, "one row of 16 lanes per group");
    if (!gany<64>(act, 0)) return false;
    bool fail = false;
    double sig = 1.0;
    invert_g16_steps<NJ, 0>(g, N, i, act, fail, sig);
    if (act) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) g[j] *= sig;
    }
    return fail;
}

// Dispatch on the group width: DPP row broadcasts for 16 lanes, LDS buffers
// (rb0, rb1, xb) for 32.
template <int NP, int NJ>
__device__ __forceinline__ bool factor_c(float2 (&m)[NJ], float mu, int N, int i, bool act, float2* rb0, float2* rb1) {
    if constexpr (NP == 16) return invert_c16<NJ>(m, mu, N, i, act);
    else return invert_c<NJ>(m, mu, N, i, act, rb0, rb1);
}

template <int NP, int NJ>
__device__ __forceinline__ float2 group_matvec(const float2 (&m)[NJ], float2 x, int i, float2* xb) {
    if constexpr (NP == 16) {
        float2 y = make_float2(0.f, 0.f);
        matvec16_steps<NJ, 0>(m, x, y);
        return y;
    } else {
        return matvec<NJ>(m, x, i, xb);
    }
}

template <int NP, int NJ>
__device__ __forceinline__ float2 group_matvec_lds(const float2* brow, float2 x, int i, float2* xb) {
    if constexpr (NP == 16) {
        float2 y = make_float2(0.f, 0.f);
        matvec16_lds_steps<NJ, 0>(brow, x, y);
        return y;
    } else {
        return matvec_lds<NJ>(brow, x, i, xb);
    }
}

// In-place FP64 Gauss-Jordan inversion of G (row i = this lane's g[]) for
// lanes with act; returns (per group) whether some pivot was <= 1e-6 or not
// finite, i.e. the inversion failed.  Same scheme as invert_c.
template <int NJ>
__device__ __forceinline__ bool invert_g(double (&g)[NJ], int N, int i, bool act, double* rbd0, double* rbd1) {
    bool fail = false;
    if (!gany<64>(act, 0)) return false;
    double sig = 1.0;
    if (act && i == 0) publish_d<NJ>(g, 0, rbd0, sig);
#pragma unroll NJ
    for (int k = 0; k < NJ; ++k) {
        if (k < N) {
            const double* buf = (k & 1) ? rbd1 : rbd0;
            double* nbuf = (k & 1) ? rbd0 : rbd1;
            if (act) {
                const double p = buf[NJ];
                fail = fail || !(p > kTauPivot && p <= 1.7976931348623157e308);
                if (i != k) {
                    const double f = g[k] * buf[NJ + 1];
                    g[k] = 0.0;
#pragma unroll
                    for (int j = 0; j < NJ; ++j) g[j] = fma(-f, buf[j], g[j]);
                }
                if (k + 1 < N && i == k + 1) publish_d<NJ>(g, (k + 1 < NJ ? k + 1 : NJ - 1), nbuf, sig);
            }
        }
    }
    if (act) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) g[j] *= sig;
    }
    return fail;
}

template <int NP, int NJ>
__device__ __forceinline__ bool factor_g(double (&g)[NJ], int N, int i, bool act, double* rb0, double* rb1) {
    if constexpr (NP == 16) return invert_g16<NJ>(g, N, i, act);
    else return invert_g<NJ>(g, N, i, act, rb0, rb1);
}

// Eigenvector of the smallest eigenvalue of the Hermitian B (this lane's
// row in LDS at bme[j * kBlock]) by shifted inverse iteration starting from
// x (unit norm).  On return m holds
// (B - mu I)^{-1} for the last accepted shift, x the unit eigenvector
// component of this lane.
//
// Every iterate is rotated by the phase of x^H y so that it keeps the phase
// of the previous one.  In FP32 the computed inverse is not exactly
// Hermitian, so its dominant eigenvalue carries a small phase; without the
// rotation each step turns the converged vector by that phase and the step
// length never falls below the tolerance.
template <int NP, int NJ>
__device__ __forceinline__ void eig_min(float2 (&m)[NJ], const float2* bme, float bnorm2, float mu, bool solve,
                        int N, int i, float2* rbc0, float2* rbc1, float2* xb, float2& x,
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
            const bool ok = factor_c<NP, NJ>(m, mu_req, N, i, need, rbc0, rbc1);
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
        float2 y = group_matvec<NP, NJ>(m, x, i, xb);
        const float n2 = gsum<NP>(y.x * y.x + y.y * y.y);
        const float sr = gsum<NP>(x.x * y.x + x.y * y.y);  // s = x^H y
        const float si = gsum<NP>(x.x * y.y - x.y * y.x);
        const float s2 = sr * sr + si * si;
        // scale by conj(s) / (|s| ||y||); plain 1/||y|| if s vanishes
        const bool gauge = s2 > 1e-30f * n2;
        // 1 / (||y|| |s|) as a product of two reciprocal square roots (about 1
        // ulp each), which cannot overflow where n2 * s2 would
        const float sc = __builtin_amdgcn_rsqf(n2) * (gauge ? __builtin_amdgcn_rsqf(s2) : 1.0f);
        const float2 u = gauge ? make_float2(sr * sc, -si * sc) : make_float2(sc, 0.f);
        y = cmul(y, u);
        const float dx = y.x - x.x, dy = y.y - x.y;
        const float d2 = gsum<NP>(dx * dx + dy * dy);
        const bool finite = n2 > 0.f && n2 <= 3.4e38f;
        // slow contraction: |dx| shrank by less than kRefineRate over the
        // last step (always true until two steps are known)
        const bool slow_rate = !(d2prev > 0.f) || d2 > kRefineRate * kRefineRate * d2prev;
        if (!conv) {
            if (finite) x = y;
            // converged: the step is below the tolerance, or the iteration
            // contracts at rate q < 1/2 and the remaining error, at most
            // |dx| q / (1 - q) <= 2 |dx| q, is below 2e-6:
            // d2 < d2prev / 4 and d2 * q^2 = d2^2 / d2prev < (1e-6)^2
            if (d2 < kTol2 || !finite) conv = true;
            else if (d2prev > 0.f && d2 < 0.25f * d2prev && d2 * d2 < 1e-12f * d2prev) conv = true;
            d2prev = d2;
        }
        ++it;
        if (it == 4 || it == 8 || it == 12 || it == 18) {
            // slow contraction: move the shift towards lambda_min.  The first
            // candidate rho - ||Bx - rho x|| bounds the eigenvalue nearest rho
            // from below; while x still mixes several eigenvectors it can lie
            // above lambda_min, so larger margins follow if the inertia check
            // rejects it.
            const bool slow = !conv && slow_rate;
            if (gany<64>(slow, 0)) {
                const float2 bx = group_matvec_lds<NP, NJ>(bme, x, i, xb);
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
