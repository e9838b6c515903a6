// Device building blocks of the per-pixel eigen-solve shared by the phase
// linking kernel and its adjoint: group reductions, FP64 and complex FP32
// Gauss-Jordan inversion, the matrix-core sweep that inverts one pixel's
// shifted matrix for two-row groups, and shifted inverse iteration for the
// smallest eigenpair of a Hermitian matrix.
//
// A group of NP lanes (inside one wavefront) owns one pixel, NJ >= N
// columns per row.  Two forms:
//  - 16 lanes (one DPP row), R = 1 or 2 rows per lane (rows l, l + 16): the
//    pivot row of a step and the iterate of a mat-vec are broadcast by DPP
//    row_newbcast, folded into the FMAs; no LDS traffic.  The linking kernel
//    uses it for every N, the adjoint for N <= 16.
//  - 32 lanes, one row per lane (the adjoint for N > 16): exchanges through a
//    few hundred bytes of LDS per group, one round trip per step.  LDS
//    operations of one wavefront execute in program order, so exchanges
//    within a group need no barrier.
#pragma once
#include <cmath>
#include <type_traits>

#include "internal.hpp"
#include "lanes.hpp"

namespace plk {
namespace {

constexpr double kTauPivot = 1e-6;
constexpr float kTol2 = 4e-12f;  // squared change of the unit iterate at convergence
constexpr int kMaxIter = 96;
constexpr float kRefineRate = 0.5f;           // refine the shift when |dx| shrinks slower
__constant__ float kRefine[3] = {1.f, 2.f, 4.f};  // margins of the refined shifts, in residuals
// Opaque copies of an integer: offsets formed from them are neither merged
// with earlier ones nor hoisted above this point (out of a loop), so loads
// through them are not hoisted either (which would keep the loaded values
// live in registers).
__device__ __forceinline__ int opaque_int(int v) {
    asm volatile("" : "+v"(v));
    return v;
}
// the same for a wave-uniform value, kept in a scalar register
__device__ __forceinline__ int opaque_uniform(int v) {
    asm volatile("" : "+s"(v));
    return v;
}

// Marks four loaded values as used here.  Loads whose values are first used
// under a select can be turned into a branch per load (each then waits for
// its data before the next is issued); placed after a run of loads, this
// keeps them unconditional and back to back, with one wait before it.
__device__ __forceinline__ void issued(float2& a, float2& b, float2& c, float2& d) {
    asm volatile("" : "+v"(a.x), "+v"(a.y), "+v"(b.x), "+v"(b.y), "+v"(c.x), "+v"(c.y), "+v"(d.x), "+v"(d.y));
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

// |z| of an FP32 complex value to about 2e-14 relative, without the FP64
// square-root sequence: the sum of squares in FP64 (the products are exact),
// the hardware FP64 reciprocal square root (about 2^-23 relative error) as a
// seed, and one Newton step for the square root, s (1 - (x y^2 - 1) / 2),
// whose error is 1.5 times the seed's squared.  A nonzero sum lies in
// [2^-298, 2^257), inside the seed's range; zero gives zero (its seed is
// taken at 1e-300), so there is no branch and no select.
__device__ __forceinline__ double cabs64(float re, float im) {
    const double x = fma((double)re, (double)re, (double)im * (double)im);
    const double y = __builtin_amdgcn_rsq(fmax(x, 1e-300));
    const double s = x * y;
    return fma(s, fma(-s, 0.5 * y, 0.5), s);
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

// ---- 16-lane groups: exchanges by DPP row broadcast.  A group of 16 lanes
// is one DPP row, and row_newbcast:L hands lane L's register to every lane of
// the row inside the instruction's operand path.  The pivot row of a
// Gauss-Jordan step (held by its owner lane) and the iterate of a mat-vec
// (R components per lane) then move between lanes without LDS traffic or its
// round-trip latency.  Lane l holds the R rows l, l + 16, ... (R = 1 for
// N <= 16, R = 2 for N <= 32), so row k lives in lane k % 16, slot k / 16.
// For R = 1 the arithmetic, and its order, is that of the LDS versions above.
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
// 1/p itself; the owner keeps row K as S_K with the diagonal slot set to 1,
// every other row i of an active group subtracts (S_i[K] / p) S_K.
// Four columns of a complex Gauss-Jordan step with the pivot-row broadcast
// folded into the FMAs (v_fmac_f32_dpp with row_newbcast:KL; negated terms
// use the instruction's negate modifier on the broadcast operand), so no
// separate broadcast or negation instructions are issued.  The compiler does
// not fold a broadcast into an FMA by itself.  Per entry (r_x, r_y = row K's
// entry): x = fma(-fx, r_x, fma(fy, r_y, x)) and
// y = fma(-fx, r_y, fma(-fy, r_x, y)), each a single-rounding FMA.  The four
// phases are ordered so that no broadcast read follows a write of the same
// register within two instructions (the DPP read hazard); the leading s_nop
// covers writes by the code just before the block.  Only the pivot lane's
// value is ever broadcast, and its row is left unchanged (its multipliers
// are zero).
template <int R, int NJ, int KS, int KL, int J0>
__device__ __forceinline__ void gj_block(float2 (&m)[R][NJ], const float (&fy)[R], const float (&fx)[R]) {
    // wait states before the first DPP read: 2 cover a VALU write just
    // before the block; the first block of a step may follow a block
    // boundary and gets 5, which also covers a write of EXEC
    constexpr int kNop = J0 == 0 ? 4 : 1;
    if constexpr (R == 1) {
        asm volatile(
        "s_nop %c11\n\t"
        "v_fmac_f32_dpp %0, %1, %8 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %3, %8 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %4, %5, %8 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %6, %7, %8 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, -%0, %8 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, -%2, %8 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %5, -%4, %8 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %7, -%6, %8 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, -%0, %9 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, -%2, %9 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %4, -%4, %9 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %6, -%6, %9 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, -%1, %9 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, -%3, %9 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %5, -%5, %9 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %7, -%7, %9 row_newbcast:%c10 row_mask:0xf bank_mask:0xf"
            : "+v"(m[0][J0].x), "+v"(m[0][J0].y), "+v"(m[0][J0 + 1].x), "+v"(m[0][J0 + 1].y),
              "+v"(m[0][J0 + 2].x), "+v"(m[0][J0 + 2].y), "+v"(m[0][J0 + 3].x), "+v"(m[0][J0 + 3].y)
            : "v"(fy[0]), "v"(fx[0]), "i"(KL), "i"(kNop));
    } else if constexpr (KS == 0) {
        asm volatile(
        "s_nop %c21\n\t"
        "v_fmac_f32_dpp %2, %1, %18 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %6, %5, %18 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %10, %9, %18 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %14, %13, %18 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %16 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %4, %5, %16 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %8, %9, %16 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %12, %13, %16 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, -%0, %18 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %7, -%4, %18 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %11, -%8, %18 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %15, -%12, %18 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, -%0, %16 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %5, -%4, %16 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %9, -%8, %16 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %13, -%12, %16 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, -%0, %19 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %6, -%4, %19 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %10, -%8, %19 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %14, -%12, %19 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, -%0, %17 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %4, -%4, %17 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %8, -%8, %17 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %12, -%12, %17 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, -%1, %19 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %7, -%5, %19 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %11, -%9, %19 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %15, -%13, %19 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, -%1, %17 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %5, -%5, %17 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %9, -%9, %17 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %13, -%13, %17 row_newbcast:%c20 row_mask:0xf bank_mask:0xf"
            : "+v"(m[0][J0].x), "+v"(m[0][J0].y), "+v"(m[1][J0].x), "+v"(m[1][J0].y),
              "+v"(m[0][J0 + 1].x), "+v"(m[0][J0 + 1].y), "+v"(m[1][J0 + 1].x), "+v"(m[1][J0 + 1].y),
              "+v"(m[0][J0 + 2].x), "+v"(m[0][J0 + 2].y), "+v"(m[1][J0 + 2].x), "+v"(m[1][J0 + 2].y),
              "+v"(m[0][J0 + 3].x), "+v"(m[0][J0 + 3].y), "+v"(m[1][J0 + 3].x), "+v"(m[1][J0 + 3].y)
            : "v"(fy[0]), "v"(fx[0]), "v"(fy[1]), "v"(fx[1]), "i"(KL), "i"(kNop));
    } else {
        asm volatile(
        "s_nop %c21\n\t"
        "v_fmac_f32_dpp %0, %3, %16 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %4, %7, %16 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %8, %11, %16 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %12, %15, %16 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %3, %18 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %6, %7, %18 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %10, %11, %18 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %14, %15, %18 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, -%2, %16 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %5, -%6, %16 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %9, -%10, %16 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %13, -%14, %16 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, -%2, %18 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %7, -%6, %18 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %11, -%10, %18 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %15, -%14, %18 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, -%2, %17 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %4, -%6, %17 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %8, -%10, %17 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %12, -%14, %17 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, -%2, %19 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %6, -%6, %19 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %10, -%10, %19 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %14, -%14, %19 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, -%3, %17 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %5, -%7, %17 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %9, -%11, %17 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %13, -%15, %17 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, -%3, %19 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %7, -%7, %19 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %11, -%11, %19 row_newbcast:%c20 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %15, -%15, %19 row_newbcast:%c20 row_mask:0xf bank_mask:0xf"
            : "+v"(m[0][J0].x), "+v"(m[0][J0].y), "+v"(m[1][J0].x), "+v"(m[1][J0].y),
              "+v"(m[0][J0 + 1].x), "+v"(m[0][J0 + 1].y), "+v"(m[1][J0 + 1].x), "+v"(m[1][J0 + 1].y),
              "+v"(m[0][J0 + 2].x), "+v"(m[0][J0 + 2].y), "+v"(m[1][J0 + 2].x), "+v"(m[1][J0 + 2].y),
              "+v"(m[0][J0 + 3].x), "+v"(m[0][J0 + 3].y), "+v"(m[1][J0 + 3].x), "+v"(m[1][J0 + 3].y)
            : "v"(fy[0]), "v"(fx[0]), "v"(fy[1]), "v"(fx[1]), "i"(KL), "i"(kNop));
    }
}

template <int R, int NJ, int KS, int KL, int J0>
__device__ __forceinline__ void gj_blocks(float2 (&m)[R][NJ], const float (&fy)[R], const float (&fx)[R]) {
    if constexpr (J0 < NJ) {
        gj_block<R, NJ, KS, KL, J0>(m, fy, fx);
        gj_blocks<R, NJ, KS, KL, J0 + 4>(m, fy, fx);
    }
}

// Step K of the complex Gauss-Jordan inversion of (m - mu I) with deferred
// row scaling: every lane reads the pivot p = m_K[K] - mu and forms 1/p
// itself; the owner keeps row K as S_K with the diagonal slot set to 1, every
// other row i subtracts (S_i[K] / p) S_K.  Every group of the wavefront
// factors (with its own shift): a per-group "skip" flag would turn the
// updates into selects that keep two copies of the matrix live.
template <int R, int NJ, int K>
__device__ __forceinline__ void invert_cr_step(float2 (&m)[R][NJ], float mu, int l, bool& pd, float (&sig)[R]) {
    constexpr int KL = K % 16, KS = K / 16;  // owner lane and slot of row K
    const float p = rowcast<KL>(m[KS][K].x) - mu;
    pd = pd && (p > 0.f) && (p <= 3.4e38f);
    const float rp = __builtin_amdgcn_rcpf(p);
    float fx[R], fy[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool piv = r == KS && l == KL;
        sig[r] = piv ? rp : sig[r];
        fx[r] = piv ? 0.f : m[r][K].x * rp;
        fy[r] = piv ? 0.f : m[r][K].y * rp;
        m[r][K] = make_float2(piv ? 1.f : 0.f, 0.f);
    }
    static_assert(NJ % 4 == 0, "columns in blocks of four");
    // for every column j and row r, with (r_x, r_y) = row K's entry j:
    //   m[r][j].x = fma(-fx, r_x, fma(fy, r_y, m[r][j].x))
    //   m[r][j].y = fma(-fx, r_y, fma(-fy, r_x, m[r][j].y))
    gj_blocks<R, NJ, KS, KL, 0>(m, fy, fx);
}

// Smallest N served by the NJ-column kernels (NJ = 12 serves every N up to
// 12, the wider ones N rounded up to a multiple of 4): steps below it always
// lie inside N and need no guard (guarding every step splits m's live ranges
// at each join).
template <int NJ>
constexpr int kMinN = NJ <= 12 ? 1 : NJ - 3;

// Steps K onwards; those at or beyond kMinN are guarded by a uniform K < N.
template <int R, int NJ, int K>
__device__ __forceinline__ void invert_cr_steps(float2 (&m)[R][NJ], float mu, int N, int l, bool& pd,
                                                float (&sig)[R]) {
    if constexpr (K < NJ) {
        if constexpr (K < kMinN<NJ>) {
            invert_cr_step<R, NJ, K>(m, mu, l, pd, sig);
        } else {
            if (K < N) invert_cr_step<R, NJ, K>(m, mu, l, pd, sig);
        }
        invert_cr_steps<R, NJ, K + 1>(m, mu, N, l, pd, sig);
    }
}

// In-place inversion of (m - mu I) for every group of the wavefront; returns
// (per group) whether every pivot was positive and finite (Sylvester's
// inertia: mu < lambda_min).
template <int R, int NJ>
__device__ __forceinline__ bool invert_cr(float2 (&m)[R][NJ], float mu, int N, int l) {
    static_assert(NJ <= 16 * R, "R rows of 16 lanes per group");
    bool pd = true;
    float sig[R];
#pragma unroll
    for (int r = 0; r < R; ++r) sig[r] = 1.f;
    invert_cr_steps<R, NJ, 0>(m, mu, N, l, pd, sig);
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < NJ; ++j) m[r][j] = make_float2(m[r][j].x * sig[r], m[r][j].y * sig[r]);
    return pd;
}


// y += B x over columns J onwards, B's row in LDS element-major (one row per lane)
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

// Four columns of an FP64 Gauss-Jordan step with the pivot-row broadcast
// folded into v_fmac_f64_dpp (row_newbcast, negate modifier on the broadcast
// operand), g[r][j] = fma(-f[r], b, g[r][j]) with b = row K's entry j.  Within a block no instruction reads a register
// written by an earlier one (the row holding row K goes last), so only the
// leading s_nop is needed for the DPP read hazard.
template <int R, int NJ, int KS, int KL, int J0>
__device__ __forceinline__ void gjd_block(double (&g)[R][NJ], const double (&f)[R]) {
    constexpr int kNop = J0 == 0 ? 4 : 1;
    if constexpr (R == 1) {
        asm volatile(
        "s_nop %c6\n\t"
        "v_fmac_f64_dpp %0, -%0, %4 row_newbcast:%c5 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %1, -%1, %4 row_newbcast:%c5 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %2, -%2, %4 row_newbcast:%c5 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %3, -%3, %4 row_newbcast:%c5 row_mask:0xf bank_mask:0xf"
            : "+v"(g[0][J0]), "+v"(g[0][J0 + 1]), "+v"(g[0][J0 + 2]), "+v"(g[0][J0 + 3])
            : "v"(f[0]), "i"(KL), "i"(kNop));
    } else if constexpr (KS == 0) {
        asm volatile(
        "s_nop %c11\n\t"
        "v_fmac_f64_dpp %1, -%0, %9 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %3, -%2, %9 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %5, -%4, %9 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %7, -%6, %9 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %0, -%0, %8 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %2, -%2, %8 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %4, -%4, %8 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %6, -%6, %8 row_newbcast:%c10 row_mask:0xf bank_mask:0xf"
            : "+v"(g[0][J0]), "+v"(g[1][J0]), "+v"(g[0][J0 + 1]), "+v"(g[1][J0 + 1]),
              "+v"(g[0][J0 + 2]), "+v"(g[1][J0 + 2]), "+v"(g[0][J0 + 3]), "+v"(g[1][J0 + 3])
            : "v"(f[0]), "v"(f[1]), "i"(KL), "i"(kNop));
    } else {
        asm volatile(
        "s_nop %c11\n\t"
        "v_fmac_f64_dpp %0, -%1, %8 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %2, -%3, %8 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %4, -%5, %8 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %6, -%7, %8 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %1, -%1, %9 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %3, -%3, %9 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %5, -%5, %9 row_newbcast:%c10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %7, -%7, %9 row_newbcast:%c10 row_mask:0xf bank_mask:0xf"
            : "+v"(g[0][J0]), "+v"(g[1][J0]), "+v"(g[0][J0 + 1]), "+v"(g[1][J0 + 1]),
              "+v"(g[0][J0 + 2]), "+v"(g[1][J0 + 2]), "+v"(g[0][J0 + 3]), "+v"(g[1][J0 + 3])
            : "v"(f[0]), "v"(f[1]), "i"(KL), "i"(kNop));
    }
}

template <int R, int NJ, int KS, int KL, int J0>
__device__ __forceinline__ void gjd_blocks(double (&g)[R][NJ], const double (&f)[R]) {
    if constexpr (J0 < NJ) {
        gjd_block<R, NJ, KS, KL, J0>(g, f);
        gjd_blocks<R, NJ, KS, KL, J0 + 4>(g, f);
    }
}

template <int R, int NJ, int K>
__device__ __forceinline__ void invert_gr_step(double (&g)[R][NJ], int l, bool& fail, double (&sig)[R]) {
    constexpr int KL = K % 16, KS = K / 16;
    const double p = rowcast<KL>(g[KS][K]);
    fail = fail || !(p > kTauPivot && p <= 1.7976931348623157e308);
    double rp = __builtin_amdgcn_rcp(p);
    rp = fma(rp, fma(-p, rp, 1.0), rp);
    rp = fma(rp, fma(-p, rp, 1.0), rp);
    double f[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool piv = r == KS && l == KL;
        sig[r] = piv ? rp : sig[r];
        f[r] = piv ? 0.0 : g[r][K] * rp;
        g[r][K] = piv ? 1.0 : 0.0;
    }
    // g[r][j] = fma(-f[r], v, g[r][j]) for every column j, v = row K's entry j.
    // (With one row per lane the blocks' register constraints cost a
    // wavefront per SIMD, and the saved broadcast moves still win: the
    // kernel is bound by instruction issue.)
    gjd_blocks<R, NJ, KS, KL, 0>(g, f);
}

template <int R, int NJ, int K>
__device__ __forceinline__ void invert_gr_steps(double (&g)[R][NJ], int N, int l, bool& fail, double (&sig)[R]) {
    if constexpr (K < NJ) {
        if constexpr (K < kMinN<NJ>) {
            invert_gr_step<R, NJ, K>(g, l, fail, sig);
        } else {
            if (K < N) invert_gr_step<R, NJ, K>(g, l, fail, sig);
        }
        invert_gr_steps<R, NJ, K + 1>(g, N, l, fail, sig);
    }
}

// In-place FP64 inversion of G for every group of the wavefront; returns
// (per group) whether some pivot was <= 1e-6 or not finite.
template <int R, int NJ>
__device__ __forceinline__ bool invert_gr(double (&g)[R][NJ], int N, int l) {
    static_assert(NJ <= 16 * R, "R rows of 16 lanes per group");
    bool fail = false;
    double sig[R];
#pragma unroll
    for (int r = 0; r < R; ++r) sig[r] = 1.0;
    invert_gr_steps<R, NJ, 0>(g, N, l, fail, sig);
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < NJ; ++j) g[r][j] *= sig[r];
    return fail;
}

// ---- Dispatch on the group width: DPP row broadcasts for 16 lanes (R rows
// per lane), LDS buffers (rb0, rb1, xb) for 32 lanes (one row per lane).
template <int NP, int R, int NJ>
__device__ __forceinline__ bool factor_c(float2 (&m)[R][NJ], float mu, int N, int i, bool act, float2* rb0,
                                         float2* rb1) {
    if constexpr (NP == 16) return invert_cr<R, NJ>(m, mu, N, i);  // every group factors
    else return invert_c<NJ>(m[0], mu, N, i, act, rb0, rb1);
}

// y += M x over four columns with the broadcast of x_j (from lane j % 16)
// folded into v_fmac_f32_dpp.  Columns in order, and per column and
// accumulator: y.x = fma(m.x, x_x, fma(-m.y, x_y, y.x)) and
// y.y = fma(m.x, x_y, fma(m.y, x_x, y.y)).  The broadcast source x is not
// written inside the block.
template <int R, int NJ, int J0>
__device__ __forceinline__ void matvec_block(const float2 (&m)[R][NJ], const float2 (&x)[R], float2 (&y)[R]) {
    constexpr int kNop = J0 == 0 ? 4 : 1;
    constexpr int S = J0 / 16;  // slot of x holding columns J0 .. J0 + 3
    if constexpr (R == 1) {
        asm volatile(
        "s_nop %c16\n\t"
        "v_fmac_f32_dpp %0, -%3, %5 row_newbcast:%c12 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %2, %5 row_newbcast:%c12 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %2, %4 row_newbcast:%c12 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %3, %4 row_newbcast:%c12 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, -%3, %7 row_newbcast:%c13 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %2, %7 row_newbcast:%c13 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %2, %6 row_newbcast:%c13 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %3, %6 row_newbcast:%c13 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, -%3, %9 row_newbcast:%c14 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %2, %9 row_newbcast:%c14 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %2, %8 row_newbcast:%c14 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %3, %8 row_newbcast:%c14 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, -%3, %11 row_newbcast:%c15 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %2, %11 row_newbcast:%c15 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %2, %10 row_newbcast:%c15 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %3, %10 row_newbcast:%c15 row_mask:0xf bank_mask:0xf"
            : "+v"(y[0].x), "+v"(y[0].y)
            : "v"(x[S].x), "v"(x[S].y), "v"(m[0][J0].x), "v"(m[0][J0].y), "v"(m[0][J0 + 1].x), "v"(m[0][J0 + 1].y),
              "v"(m[0][J0 + 2].x), "v"(m[0][J0 + 2].y), "v"(m[0][J0 + 3].x), "v"(m[0][J0 + 3].y),
              "i"(J0 % 16), "i"((J0 + 1) % 16), "i"((J0 + 2) % 16), "i"((J0 + 3) % 16), "i"(kNop));
    } else {
        asm volatile(
        "s_nop %c26\n\t"
        "v_fmac_f32_dpp %0, -%5, %7 row_newbcast:%c22 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, -%5, %9 row_newbcast:%c22 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %4, %7 row_newbcast:%c22 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %4, %9 row_newbcast:%c22 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %4, %6 row_newbcast:%c22 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %4, %8 row_newbcast:%c22 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %5, %6 row_newbcast:%c22 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %5, %8 row_newbcast:%c22 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, -%5, %11 row_newbcast:%c23 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, -%5, %13 row_newbcast:%c23 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %4, %11 row_newbcast:%c23 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %4, %13 row_newbcast:%c23 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %4, %10 row_newbcast:%c23 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %4, %12 row_newbcast:%c23 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %5, %10 row_newbcast:%c23 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %5, %12 row_newbcast:%c23 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, -%5, %15 row_newbcast:%c24 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, -%5, %17 row_newbcast:%c24 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %4, %15 row_newbcast:%c24 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %4, %17 row_newbcast:%c24 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %4, %14 row_newbcast:%c24 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %4, %16 row_newbcast:%c24 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %5, %14 row_newbcast:%c24 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %5, %16 row_newbcast:%c24 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, -%5, %19 row_newbcast:%c25 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, -%5, %21 row_newbcast:%c25 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %4, %19 row_newbcast:%c25 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %4, %21 row_newbcast:%c25 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %4, %18 row_newbcast:%c25 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %4, %20 row_newbcast:%c25 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %5, %18 row_newbcast:%c25 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %5, %20 row_newbcast:%c25 row_mask:0xf bank_mask:0xf"
            : "+v"(y[0].x), "+v"(y[0].y), "+v"(y[1].x), "+v"(y[1].y)
            : "v"(x[S].x), "v"(x[S].y),
              "v"(m[0][J0].x), "v"(m[0][J0].y), "v"(m[1][J0].x), "v"(m[1][J0].y),
              "v"(m[0][J0 + 1].x), "v"(m[0][J0 + 1].y), "v"(m[1][J0 + 1].x), "v"(m[1][J0 + 1].y),
              "v"(m[0][J0 + 2].x), "v"(m[0][J0 + 2].y), "v"(m[1][J0 + 2].x), "v"(m[1][J0 + 2].y),
              "v"(m[0][J0 + 3].x), "v"(m[0][J0 + 3].y), "v"(m[1][J0 + 3].x), "v"(m[1][J0 + 3].y),
              "i"(J0 % 16), "i"((J0 + 1) % 16), "i"((J0 + 2) % 16), "i"((J0 + 3) % 16), "i"(kNop));
    }
}

template <int R, int NJ, int J0>
__device__ __forceinline__ void matvec_blocks(const float2 (&m)[R][NJ], const float2 (&x)[R], float2 (&y)[R]) {
    if constexpr (J0 < NJ) {
        matvec_block<R, NJ, J0>(m, x, y);
        matvec_blocks<R, NJ, J0 + 4>(m, x, y);
    }
}

template <int NP, int R, int NJ>
__device__ __forceinline__ void group_matvec(const float2 (&m)[R][NJ], const float2 (&x)[R], float2 (&y)[R], int i,
                                             float2* xb) {
    if constexpr (NP == 16) {
#pragma unroll
        for (int r = 0; r < R; ++r) y[r] = make_float2(0.f, 0.f);
        matvec_blocks<R, NJ, 0>(m, x, y);
    } else {
        y[0] = matvec<NJ>(m[0], x[0], i, xb);
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

template <int NP, int R, int NJ>
__device__ __forceinline__ bool factor_g(double (&g)[R][NJ], int N, int i, bool act, double* rb0, double* rb1) {
    if constexpr (NP == 16) {
        if (!gany<64>(act, 0)) return false;
        return invert_gr<R, NJ>(g, N, i) && act;  // every group factors; failures count where act
    }
    else return invert_g<NJ>(g[0], N, i, act, rb0, rb1);
}

// ---- Where the Hermitian B of a group lives between factorisations.
//
// BRowLds: each lane's row, element-major over the workgroup (element j of
// the row at p[j * kBlock]), so the lanes of a wavefront touch consecutive
// words.  One row per lane.
template <int NP, int NJ>
struct BRowLds {
    float2* p;
    float2* xb;  // iterate buffer of the group (32-lane groups)
    int i;
    // the row is read through an opaque zero offset, so that the loads stay
    // inside the solver loop (nothing in the loop writes LDS, and hoisted
    // they would occupy NJ register pairs next to m)
    __device__ __forceinline__ void load(float2 (&m)[1][NJ], bool pred) const {
        if (pred) {
            const float2* q = p + opaque_int(0);
#pragma unroll
            for (int j = 0; j < NJ; ++j) m[0][j] = q[j * kBlock];
        }
    }
    __device__ __forceinline__ void apply(const float2 (&x)[1], float2 (&y)[1]) const {
        y[0] = group_matvec_lds<NP, NJ>(p + opaque_int(0), x[0], i, xb);
    }
};

// BTriLds: two rows per lane (N <= 32); the upper triangle of each group's
// matrix (the lower part is its conjugate), so that three wavefronts per
// SIMD fit in LDS.  Entry (a, b >= a) has index a (2 NJ - a - 1) / 2 + b and
// the four groups of a wavefront interleave: entry e of group g at
// w[e * 4 + g].  Index TRI of each group is a write sink for the stores of
// entries a lane does not own, so that stores need no branch.
//
// Offsets: row i's upper entries (i, j >= i) lie at up_i + 4 j, and its
// lower entries (j < i), read as entry (j, i), at lo_i + 4 cj(j) with
// cj(j) = j (2 NJ - j - 1) / 2 a compile-time constant, so every access is a
// per-lane base plus an immediate.  A read loads both candidates and keeps
// the one on its side of the diagonal; bases are clamped so that both stay
// inside the buffer.
template <int NJ>
struct BTriLds {
    static constexpr int TRI = NJ * (NJ + 1) / 2;
    static constexpr int GPW = 4;
    static constexpr int WAVE_ENTRIES = (TRI + 1) * GPW;  // float2 per wavefront
    static constexpr int cj(int j) { return j * (2 * NJ - j - 1) / 2; }
    float2* w;  // this wavefront's buffer
    int g, l, N;
    float2* xs;  // this wavefront's 16 x 33 scratch for matrix-core factorisations

    __device__ __forceinline__ int up_base(int ll, int r) const {
        const int i = ll + 16 * r;
        return (i * (2 * NJ - i - 1) / 2) * GPW + g;
    }
    __device__ __forceinline__ int lo_base(int ll, int r) const {
        const int i = min(ll + 16 * r, NJ - 1);
        return i * GPW + g;
    }
    __device__ __forceinline__ int sink() const { return TRI * GPW + g; }

    // B[ll + 16 r][J]; zero outside n x n.  The entry's offset is selected
    // first and read with one load (selecting between two loaded values
    // lets the compiler put each load in a branch of its own, with a wait).
    template <int J>
    __device__ __forceinline__ int offset(int ub, int lb, int ll, int r) const {
        return J >= ll + 16 * r ? ub + J * GPW : lb + cj(J) * GPW;  // entry (i, J), or (J, i) below the diagonal
    }
    // B[i][J] from the stored entry v read at offset<J>()
    template <int J>
    __device__ __forceinline__ float2 entry(float2 v, int ll, int r, int n) const {
        const int i = ll + 16 * r;
        const float2 h = make_float2(v.x, J >= i ? v.y : -v.y);
        return (i < n && J < n) ? h : make_float2(0.f, 0.f);
    }
    template <int J>
    __device__ __forceinline__ float2 get(int ub, int lb, int ll, int r, int n) const {
        return entry<J>(w[offset<J>(ub, lb, ll, r)], ll, r, n);
    }
    // offset of entry (i, J) if this lane owns it (J >= i, both < N), else the sink
    template <int J>
    __device__ __forceinline__ int own(int ub, int ll, int r, int n) const {
        const int i = ll + 16 * r;
        return (J >= i && i < n && J < n) ? ub + J * GPW : sink();
    }

    template <int J>
    __device__ __forceinline__ void load_steps(float2 (&m)[2][NJ], const int (&ub)[2], const int (&lb)[2], int ll,
                                               int n) const {
        if constexpr (J < NJ) {
#pragma unroll
            for (int r = 0; r < 2; ++r) m[r][J] = get<J>(ub[r], lb[r], ll, r, n);
            load_steps<J + 1>(m, ub, lb, ll, n);
        }
    }
    // one branch around the whole reload: the loads of the lanes with pred
    // write m in place (a select per entry would keep both copies live).
    // The lane index and N are taken through opaque copies so that the
    // offsets are formed here rather than kept live across the solver loop.
    __device__ __forceinline__ void load(float2 (&m)[2][NJ], bool pred) const {
        if (pred) {
            const int ll = opaque_int(l), n = opaque_uniform(N);
            __builtin_assume(n >= kMinN<NJ> && n <= NJ);
            const int ub[2] = {up_base(ll, 0), up_base(ll, 1)}, lb[2] = {lo_base(ll, 0), lo_base(ll, 1)};
            load_steps<0>(m, ub, lb, ll, n);
        }
    }
    // Columns J .. J + 3: the eight entries are loaded before any is used, so
    // that one wait covers them (used one by one, each load would wait for
    // its data before the next is issued); at most four columns in flight,
    // since all of them would need 8 NJ registers next to the factorisation.
    template <int J>
    __device__ __forceinline__ void apply_steps(const int (&ub)[2], const int (&lb)[2], int ll, int n,
                                                const float2 (&x)[2], float2 (&y)[2]) const {
        if constexpr (J < NJ) {
            float2 b[4][2];
            [&]<int... Q>(std::integer_sequence<int, Q...>) {
                ((b[Q][0] = w[offset<J + Q>(ub[0], lb[0], ll, 0)], b[Q][1] = w[offset<J + Q>(ub[1], lb[1], ll, 1)]),
                 ...);
            }(std::make_integer_sequence<int, 4>{});
            issued(b[0][0], b[0][1], b[1][0], b[1][1]);
            issued(b[2][0], b[2][1], b[3][0], b[3][1]);
            [&]<int... Q>(std::integer_sequence<int, Q...>) {
                ((b[Q][0] = entry<J + Q>(b[Q][0], ll, 0, n), b[Q][1] = entry<J + Q>(b[Q][1], ll, 1, n)), ...);
            }(std::make_integer_sequence<int, 4>{});
            [&]<int... Q>(std::integer_sequence<int, Q...>) {
                auto col = [&](auto qc) __attribute__((always_inline)) {
                    constexpr int q = decltype(qc)::value;
                    const float vx = rowcast<(J + q) % 16>(x[(J + q) / 16].x), vy = rowcast<(J + q) % 16>(x[(J + q) / 16].y);
#pragma unroll
                    for (int r = 0; r < 2; ++r) {
                        y[r].x = fmaf(b[q][r].x, vx, fmaf(-b[q][r].y, vy, y[r].x));
                        y[r].y = fmaf(b[q][r].x, vy, fmaf(b[q][r].y, vx, y[r].y));
                    }
                };
                (col(std::integral_constant<int, Q>{}), ...);
            }(std::make_integer_sequence<int, 4>{});
            __builtin_amdgcn_sched_barrier(0);
            apply_steps<J + 4>(ub, lb, ll, n, x, y);
        }
    }
    // y = B x for this lane's two rows
    __device__ __forceinline__ void apply(const float2 (&x)[2], float2 (&y)[2]) const {
        const int ll = opaque_int(l), n = opaque_uniform(N);
        __builtin_assume(n >= kMinN<NJ> && n <= NJ);
        const int ub[2] = {up_base(ll, 0), up_base(ll, 1)}, lb[2] = {lo_base(ll, 0), lo_base(ll, 1)};
        y[0] = y[1] = make_float2(0.f, 0.f);
        apply_steps<0>(ub, lb, ll, n, x, y);
    }
};

// ---- (B - mu I)^{-1} of one pixel on the matrix cores (two rows per lane,
// N <= 32).  The whole wavefront works on one 16-lane group's matrix at a
// time, held as two 32 x 32 FP32 accumulators (real and imaginary parts) in
// the layout of v_mfma_f32_32x32x2f32: lane l holds column l % 32 of rows
// acc_row(v, l / 32), v = 0..15.  Rows and columns at or beyond N are zero.
//
// Sweep operator on the Hermitian A = B - mu I: for each pivot k < N, with
// p = a_kk and r = row k,
//   a_ij <- a_ij - a_ik a_kj / p,  a_kj <- a_kj / p,  a_ik <- a_ik / p,
//   a_kk <- -1 / p,
// which keeps A Hermitian (column k is conj(row k)) and, after all pivots,
// leaves -A^{-1}.  One step is one complex rank-1 update of the whole
// matrix, two real rank-2 MFMAs: with f_i = conj(r_i) / p,
//   Re A -= [-Re f | Im f] x [Re r ; Im r],  Im A -= [-Re f | -Im f] x [Im r ; Re r]
// (A operand: lane l gives row l % 32, column l / 32; B operand: lane l gives
// row l / 32, column l % 32).  Row and column k come out of the same update
// when f_k is replaced by 1 - 1/p and r_k by p - 1, and the diagonal entry by
// first subtracting 2 from a_kk:  (p - 2) - (1 - 1/p)(p - 1) = -1/p.
// All pivots positive and finite proves mu < lambda_min(B) (Sylvester's
// inertia), as with the Gauss-Jordan form.
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ constexpr int acc_row(int v, int h) { return 8 * (v >> 2) + 4 * h + (v & 3); }

// Operands of sweep step K for one accumulator pair (VALU part).  Row K
// lives in register KV of the lanes of half KH.  v_permlane32_swap a, b
// exchanges the upper 32 lanes of a with the lower 32 lanes of b: applied to
// copies of the real and imaginary registers it leaves {Re r, Im r} in the
// copy of half KH (lane c: Re r_c, lane c + 32: Im r_c), which is exactly
// the B operand of the real update; with the operands exchanged it leaves
// {Im r, Re r}, the B operand of the imaginary update.
template <int K>
__device__ __forceinline__ void sweep_operands(f32x16& ar, f32x16& ai, int lane, float& are, float& bre,
                                               float& aim, float& bim, bool& pd) {
    constexpr int KV = 4 * (K >> 3) + (K & 3), KH = (K >> 2) & 1;
    const int c = lane & 31, h = lane >> 5;
    float x = ar[KV], y = ai[KV];
    asm volatile("s_nop 1\n\tv_permlane32_swap_b32 %0, %1\n\ts_nop 1" : "+v"(x), "+v"(y));
    bre = KH ? y : x;  // lane c: Re r_c, lane c + 32: Im r_c
    float u = ar[KV], w = ai[KV];  // the same swap with the operands exchanged
    asm volatile("s_nop 1\n\tv_permlane32_swap_b32 %0, %1\n\ts_nop 1" : "+v"(w), "+v"(u));
    bim = KH ? u : w;  // lane c: Im r_c, lane c + 32: Re r_c
    const float p = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bre), K));
    pd = pd && (p > 0.f) && (p <= 3.4e38f);
    const float rp = __builtin_amdgcn_rcpf(p);
    are = -bre * rp;          // -Re f_c (lane c), Im f_c (lane c + 32); f_c = conj(r_c) / p
    aim = h ? -are : are;     // -Re f_c, -Im f_c
    if (c == K) {
        const float phi = 1.f - rp, rho = p - 1.f;
        are = h ? 0.f : -phi;
        aim = are;
        bre = h ? 0.f : rho;
        bim = h ? rho : 0.f;
    }
}

// Steps K onwards for one (TWO = false) or two independent matrices; each
// matrix's MFMAs are issued before the other's operands are formed, so that
// they overlap each other's latency (scheduling barriers keep that order).
template <int NJ, int K, bool TWO>
__device__ __forceinline__ void sweep_steps(f32x16& ar0, f32x16& ai0, f32x16& ar1, f32x16& ai1, int N, int lane,
                                            bool& pd0, bool& pd1) {
    if constexpr (K < NJ) {
        constexpr int KV = 4 * (K >> 3) + (K & 3), KH = (K >> 2) & 1;
        if (K < kMinN<NJ> || K < N) {
            const float two = lane == K + 32 * KH ? 2.f : 0.f;
            float a0, b0, c0, d0;
            sweep_operands<K>(ar0, ai0, lane, a0, b0, c0, d0, pd0);
            ar0[KV] -= two;
            ar0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, ar0, 0, 0, 0);
            ai0 = __builtin_amdgcn_mfma_f32_32x32x2f32(c0, d0, ai0, 0, 0, 0);
            if constexpr (TWO) {
                __builtin_amdgcn_sched_barrier(0);
                float a1, b1, c1, d1;
                sweep_operands<K>(ar1, ai1, lane, a1, b1, c1, d1, pd1);
                ar1[KV] -= two;
                ar1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, ar1, 0, 0, 0);
                ai1 = __builtin_amdgcn_mfma_f32_32x32x2f32(c1, d1, ai1, 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        sweep_steps<NJ, K + 1, TWO>(ar0, ai0, ar1, ai1, N, lane, pd0, pd1);
    }
}

// A = B - mu I of group g in accumulator layout: entry (i, c) of the
// Hermitian matrix of the upper triangle; zero outside N x N.
template <int NJ>
__device__ __forceinline__ void acc_load(const BTriLds<NJ>& tri, int g, float mu, int N, int lane, f32x16& ar,
                                         f32x16& ai) {
    const int c = lane & 31, h = lane >> 5;
    float2 b[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int i = acc_row(v, h);
        // entry (min, max) of (i, c), clamped into the triangle (no select:
        // a selected offset becomes a branch); unused outside N x N
        const int lo = min(min(i, c), NJ - 1), hi = min(max(i, c), NJ - 1);
        const int e = ((lo * (2 * NJ - 1 - lo)) >> 1) + hi;
        b[v] = tri.w[e * BTriLds<NJ>::GPW + g];
    }
#pragma unroll
    for (int v = 0; v < 16; v += 4) issued(b[v], b[v + 1], b[v + 2], b[v + 3]);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int i = acc_row(v, h);
        const bool in = i < N && c < N;
        ar[v] = in ? b[v].x - (i == c ? mu : 0.f) : 0.f;
        ai[v] = in ? (i > c ? -b[v].y : b[v].y) : 0.f;
    }
}

// The sweep result S = -A^{-1} into the rows l, l + 16 of group g's lanes.
// S is Hermitian, so row t is the conjugate of column t, which lanes t and
// t + 32 hold: they write it conjugated into the wave's 16 x 33 scratch as
// a row (16 rows per pass), and lane t % 16 of group g reads it back.
template <int NJ>
__device__ __forceinline__ void acc_to_rows(const f32x16& ar, const f32x16& ai, int g, int lane, float2* xs,
                                            float2 (&m)[2][NJ]) {
    const int c = lane & 31, h = lane >> 5;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        wave_sync();  // the previous reads of the scratch are done
        if ((c >> 4) == s) {
#pragma unroll
            for (int v = 0; v < 16; ++v) xs[(c & 15) * 33 + acc_row(v, h)] = make_float2(ar[v], -ai[v]);
        }
        wave_sync();
        if ((lane >> 4) == g) {
            const float2* row = xs + (lane & 15) * 33;
#pragma unroll
            for (int j = 0; j < NJ; ++j) m[s][j] = row[j];
        }
    }
}

// -(B - mu I)^{-1} for every 16-lane group g of the wavefront with need
// (mu from the group's lanes), written into the rows l, l + 16 (m[0], m[1])
// of that group's lanes.  (Inverse iteration with the gauge fix gives the
// same iterates for -M as for M: the sign is a unit factor that the gauge
// rotation removes exactly.)  B is read from the packed triangle view `tri`;
// xs is the wavefront's 16 x 33 scratch.
//  - Three or four groups waiting: every group is factored, two at a time so
//    that the two matrices' MFMAs overlap each other's latency; groups
//    without a request redo their accepted shift, which reproduces their m
//    exactly (m's old contents are dead on this path).
//  - Fewer: one group at a time, the other groups' m left as it was.
// Returns, for this lane's group, whether every pivot was positive and
// finite (meaningful where need).
template <int NJ>
__device__ __forceinline__ bool factor_mfma(float2 (&m)[2][NJ], const BTriLds<NJ>& tri, float2* xs, float mu,
                                            bool need, int N) {
    static_assert(NJ <= 32, "32 x 32 accumulators");
    const uint64_t want = __ballot(need);
    int pending = (int)((want & 1ull) | ((want >> 15) & 2ull) | ((want >> 30) & 4ull) | ((want >> 45) & 8ull));
    bool ok = true;
    if (__builtin_popcount(pending) >= 3) {
        float2 t[2][NJ];  // every lane's rows are written by exactly one group's pass
#pragma unroll
        for (int q = 0; q < 4; q += 2) {
            const int lane = opaque_int(lane_id());
            const int grp = lane >> 4;
            const float mu0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mu), 16 * q));
            const float mu1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mu), 16 * q + 16));
            f32x16 ar0, ai0, ar1, ai1;
            acc_load<NJ>(tri, q, mu0, N, lane, ar0, ai0);
            acc_load<NJ>(tri, q + 1, mu1, N, lane, ar1, ai1);
            bool pd0 = true, pd1 = true;
            sweep_steps<NJ, 0, true>(ar0, ai0, ar1, ai1, N, lane, pd0, pd1);
            acc_to_rows<NJ>(ar0, ai0, q, lane, xs, t);
            acc_to_rows<NJ>(ar1, ai1, q + 1, lane, xs, t);
            if (grp == q) ok = pd0;
            if (grp == q + 1) ok = pd1;
        }
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int j = 0; j < NJ; ++j) m[r][j] = t[r][j];
        return ok;
    }
    while (pending) {  // uniform
        const int g = __builtin_ctz(pending);
        pending &= pending - 1;
        // an opaque lane index: the per-step lane predicates and offsets are
        // formed inside the loop instead of being hoisted and kept live
        const int lane = opaque_int(lane_id());
        const float mug = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mu), 16 * g));
        f32x16 ar, ai, unused0, unused1;
        acc_load<NJ>(tri, g, mug, N, lane, ar, ai);
        bool pd = true, pd1 = true;
        sweep_steps<NJ, 0, false>(ar, ai, unused0, unused1, N, lane, pd, pd1);
        acc_to_rows<NJ>(ar, ai, g, lane, xs, m);
        if ((lane >> 4) == g) ok = pd;
    }
    return ok;
}

// Eigenvector of the smallest eigenvalue of the Hermitian B (rows held as
// the view bv describes) by shifted inverse iteration starting from x (unit
// norm; R components per lane).  On return m holds (B - mu I)^{-1} for the
// last accepted shift and x the unit eigenvector components of this lane.
//
// Every iterate is rotated by the phase of x^H y so that it keeps the phase
// of the previous one.  In FP32 the computed inverse is not exactly
// Hermitian, so its dominant eigenvalue carries a small phase; without the
// rotation each step turns the converged vector by that phase and the step
// length never falls below the tolerance.
template <int NP, int R, int NJ, class BV>
__device__ __forceinline__ void eig_min_r(float2 (&m)[R][NJ], const BV& bv, float bnorm2, float mu, bool solve,
                                          int N, int i, float2* rbc0, float2* rbc1, float2* xb, float2 (&x)[R],
                                          bool& conv, int& it, int& retries) {
    // One factorisation site serves the first shift and its back-off
    // schedule, the refined shifts, and restoring the accepted shift after
    // every refined candidate was rejected.
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < NJ; ++j) m[r][j] = make_float2(0.f, 0.f);
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
            // 16-lane groups: every group of the wavefront factors; those
            // without a pending request redo their accepted shift, which
            // reproduces their inverse exactly
            bool ok;
            if constexpr (NP == 16 && R == 2 && std::is_same_v<BV, BTriLds<NJ>>) {
                // two rows per lane: per pixel on the matrix cores, only the
                // groups that wait for a factorisation
                ok = factor_mfma<NJ>(m, bv, bv.xs, need ? mu_req : mu, need, N);
            } else {
                if constexpr (NP == 16) bv.load(m, true);
                else bv.load(m, need);
                ok = factor_c<NP, R, NJ>(m, need ? mu_req : mu, N, i, need, rbc0, rbc1);
            }
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
        }
        // Iterate in the same pass once no group waits for a factorisation.
        // (Going back to the loop head after factoring, with `continue`, made
        // the compiler keep two register copies of m across the loop.)
        if (!gany<64>(need, 0)) {
            if (!gany<64>(!conv, 0) || it >= kMaxIter) break;
            float2 y[R];
            group_matvec<NP, R, NJ>(m, x, y, i, xb);
            float n2 = 0.f, sr = 0.f, si = 0.f;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                n2 += y[r].x * y[r].x + y[r].y * y[r].y;
                sr += x[r].x * y[r].x + x[r].y * y[r].y;  // s = x^H y
                si += x[r].x * y[r].y - x[r].y * y[r].x;
            }
            n2 = gsum<NP>(n2);
            sr = gsum<NP>(sr);
            si = gsum<NP>(si);
            const float s2 = sr * sr + si * si;
            // scale by conj(s) / (|s| ||y||); plain 1/||y|| if s vanishes
            const bool gauge = s2 > 1e-30f * n2;
            // 1 / (||y|| |s|) as a product of two reciprocal square roots (about 1
            // ulp each), which cannot overflow where n2 * s2 would
            const float sc = __builtin_amdgcn_rsqf(n2) * (gauge ? __builtin_amdgcn_rsqf(s2) : 1.0f);
            const float2 u = gauge ? make_float2(sr * sc, -si * sc) : make_float2(sc, 0.f);
            float d2 = 0.f;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                y[r] = cmul(y[r], u);
                const float dx = y[r].x - x[r].x, dy = y[r].y - x[r].y;
                d2 += dx * dx + dy * dy;
            }
            d2 = gsum<NP>(d2);
            const bool finite = n2 > 0.f && n2 <= 3.4e38f;
            // slow contraction: |dx| shrank by less than kRefineRate over the
            // last step (always true until two steps are known)
            const bool slow_rate = !(d2prev > 0.f) || d2 > kRefineRate * kRefineRate * d2prev;
            if (!conv) {
                if (finite) {
#pragma unroll
                    for (int r = 0; r < R; ++r) x[r] = y[r];
                }
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
                    float2 bx[R];
                    bv.apply(x, bx);
                    float rho = 0.f;
#pragma unroll
                    for (int r = 0; r < R; ++r) rho += x[r].x * bx[r].x + x[r].y * bx[r].y;
                    rho = gsum<NP>(rho);
                    float res2 = 0.f;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const float rx = bx[r].x - rho * x[r].x, ry = bx[r].y - rho * x[r].y;
                        res2 += rx * rx + ry * ry;
                    }
                    const float res = sqrtf(gsum<NP>(res2));
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
}

// One row per lane, B's rows element-major in LDS at bme[j * kBlock].
template <int NP, int NJ>
__device__ __forceinline__ void eig_min(float2 (&m)[1][NJ], float2* bme, float bnorm2, float mu, bool solve, int N,
                                        int i, float2* rbc0, float2* rbc1, float2* xb, float2 (&x)[1], bool& conv,
                                        int& it, int& retries) {
    const BRowLds<NP, NJ> bv{bme, xb, i};
    eig_min_r<NP, 1, NJ>(m, bv, bnorm2, mu, solve, N, i, rbc0, rbc1, xb, x, conv, it, retries);
}

}  // namespace
}  // namespace plk
