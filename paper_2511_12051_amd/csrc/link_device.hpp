// Device body of EMI / EVD phase linking (used by the linking kernels and by
// the single-launch batched path); see phase_link.hip for the method and the
// layout.
#pragma once
#include <cmath>
#include <utility>

#include "eig_device.hpp"

namespace plk {
namespace {

// offset of entry (i, j), i <= j, inside one pixel's matrix
__device__ __forceinline__ int centry(int packed, int N, int i, int j) {
    return packed ? ((i * (2 * N - i - 1)) >> 1) + j : i * N + j;
}

// LDS of one block of kBlock threads: one row per lane element-major (R = 1),
// or per wavefront the packed triangle and a 16 x 33 scratch (R = 2)
template <int R, int NJ>
constexpr int link_lds_bytes() {
    return R == 1 ? NJ * kBlock * 8 : (kBlock / 64) * (BTriLds<NJ>::WAVE_ENTRIES + 16 * 33) * 8;
}

// Pixel block `block` (kBlock / 64 wavefronts of four pixels); tid is the
// thread's index in the block (its wavefront tid / 64 picks the four
// pixels) and lds the block's link_lds_bytes() of LDS.  lds_wave (>= 0)
// names the wavefront slot of lds this wavefront uses instead of tid / 64,
// for callers whose wavefronts take the pixel groups of a block in any order.
template <int R, int NJ>
__device__ __forceinline__ void link_body(const LinkArgs& a, int64_t block, int tid, float2* lds,
                                          int lds_wave = -1) {
    constexpr int GPW = 4;  // 16-lane groups (pixels) per wavefront
    // NJ >= N columns are stored and updated per row (N rounded up to a
    // multiple of 4); lane l of a group holds rows l and, for R = 2, l + 16.
    // Between factorisations B lives in LDS: one row per lane element-major
    // (R = 1), or the packed upper triangle of each group's matrix (R = 2),
    // which is also where B is formed from C.
    using Tri = BTriLds<NJ>;
    // two-row groups: the triangle and a 16 x 33 scratch per wavefront for the
    // matrix-core factorisations
    constexpr int XS = 16 * 33;
    // opaque copies of the lane index and N: in a persistent loop the
    // compiler would otherwise precompute every per-step constant and
    // predicate once and keep them live (in spilled registers) across it
    const int lane = opaque_int(lane_id());
    const int l = lane & 15;
    const int grp = lane >> 4;
    const int wave = tid >> 6;
    const int slot = lds_wave >= 0 ? lds_wave : wave;  // LDS slot of this wavefront
    const int stid = (slot << 6) | (tid & 63);

    const int N = opaque_uniform(__builtin_amdgcn_readfirstlane(a.N));
    // every caller picks NJ as N rounded up to a multiple of four (N <= 12:
    // NJ = 12), so the per-column tests j < N are known true below NJ - 3
    __builtin_assume(N >= kMinN<NJ> && N <= NJ);
    const int64_t pix = (block * (kBlock / 64) + wave) * GPW + grp;
    const bool active = pix < a.npix;
    bool live[R];
#pragma unroll
    for (int r = 0; r < R; ++r) live[r] = active && l + 16 * r < N;

    // ---- rows of C (each lane reads its own rows; a variant staging the
    // wavefront's matrices through LDS with coalesced loads measured slower)
    // Loads are issued for every slot at clamped, in-bounds addresses and the
    // values selected afterwards: a load inside a per-entry branch waits for
    // its data before the next one is issued.
    const int packed = a.packed;
    const float2* mat = a.coh + (active ? pix : 0) * (int64_t)(packed ? (N * (N + 1)) >> 1 : N * N);
    const float2* src = mat + (int64_t)min(l, N - 1) * N;  // row l (clamped), full layout
    float2 c[R][NJ];
    if (R == 1 && !packed) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const float2 v = src[min(j, N - 1)];
            c[0][j] = (live[0] && j < N) ? v : make_float2(0.f, 0.f);
        }
    } else {
        // The Hermitian matrix of C's upper triangle (reading R13): entry
        // (i, j < i) is conj(C[j][i]), so that G = |C| is exactly symmetric
        // and the triangle of B (below) is consistent.
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = min(l + 16 * r, N - 1);
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const int jc = min(j, N - 1);
                float2 v = mat[centry(packed, N, min(i, jc), max(i, jc))];  // entry (min, max): no branch
                v.y = jc < i ? -v.y : v.y;
                c[r][j] = (live[r] && j < N) ? v : make_float2(0.f, 0.f);
            }
        }
    }
    bool bad = false;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < NJ; ++j) bad = bad | !(fabsf(c[r][j].x) <= 3.4e38f && fabsf(c[r][j].y) <= 3.4e38f);  // no short circuit: no branches
    const bool invalid = !active || gany<16>(bad, grp);

    // start from column ref of C: the single-reference interferogram phases
    float2 x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        x[r] = make_float2(0.f, 0.f);
#pragma unroll
        for (int j = 0; j < NJ; ++j)
            if (j == a.ref && live[r]) x[r] = c[r][j];
    }
    {
        // unit-modulus start: the phases of column ref (for consistent phases
        // the EMI eigenvector has entries of equal modulus)
        float nrm = 0.f;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float x2 = x[r].x * x[r].x + x[r].y * x[r].y;
            if (x2 > 0.f) {
                const float q = __builtin_amdgcn_rsqf(x2);
                x[r].x *= q;
                x[r].y *= q;
            }
            nrm += x[r].x * x[r].x + x[r].y * x[r].y;
        }
        nrm = gsum<16>(nrm);
        if (!(nrm > 0.f)) {
#pragma unroll
            for (int r = 0; r < R; ++r) x[r] = make_float2(l + 16 * r == a.ref ? 1.f : 0.f, 0.f);
            nrm = 1.f;
        }
        const float q = __builtin_amdgcn_rsqf(nrm);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            x[r].x *= q;
            x[r].y *= q;
        }
    }
    const Tri tri{lds + slot * Tri::WAVE_ENTRIES, grp, l, N, lds + (kBlock / 64) * Tri::WAVE_ENTRIES + slot * XS};
    if constexpr (R == 2) {
        // C's upper triangle goes to LDS now; B is formed there after step 1.
        // The fence orders these stores after the previous pixel's reads of
        // the triangle by other lanes (persistent loop).
        wave_sync();
        const int ub[2] = {tri.up_base(l, 0), tri.up_base(l, 1)};
        [&]<int... J>(std::integer_sequence<int, J...>) {
#pragma unroll
            for (int r = 0; r < R; ++r) ((tri.w[tri.template own<J>(ub[r], l, r, N)] = c[r][J]), ...);
        }(std::make_integer_sequence<int, NJ>{});
        wave_sync();
    }
    // ---- 1. FP64 inverse of G = |C|
    bool use_evd = a.method == PL_LINK_EVD;
    double gi[R][NJ];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < NJ; ++j) gi[r][j] = cabs64(c[r][j].x, c[r][j].y);  // c is zero outside N x N
    const bool do_emi = !use_evd && !invalid;
    const bool gfail = factor_g<16, R, NJ>(gi, N, l, do_emi, nullptr, nullptr);
    use_evd = use_evd || gfail;

    // ---- 2. the Hermitian matrix whose smallest eigenpair is wanted,
    // B = G^{-1} o C (EMI) or -C (EVD), and ||B||_F^2 (per lane, summed by
    // the solver)
    float bnorm2 = 0.f;
    if constexpr (R == 1) {
        // row i of C is read again (an L2 hit) rather than kept live across step 1
        const float2* src2 = src + opaque_int(0);
        const float2* mat2 = mat + opaque_int(0);
        const int i0 = min(l, N - 1);
        float2* bme = lds + stid;  // element j at bme[j * kBlock]
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            float2 cl;
            if (!packed) {
                cl = src2[min(j, N - 1)];
            } else {
                const int jc = min(j, N - 1);
                cl = mat2[centry(1, N, min(i0, jc), max(i0, jc))];
                cl.y = jc < i0 ? -cl.y : cl.y;
            }
            const float2 cj = (live[0] && j < N) ? cl : make_float2(0.f, 0.f);
            const float2 v = use_evd ? make_float2(-cj.x, -cj.y)
                                     : make_float2((float)gi[0][j] * cj.x, (float)gi[0][j] * cj.y);
            bme[j * kBlock] = v;
            bnorm2 = fmaf(v.x, v.x, fmaf(v.y, v.y, bnorm2));
        }
    } else {
        // in place over the upper triangle: each lane rewrites the entries it
        // owns (i, j >= i); off-diagonal entries count twice in ||B||_F^2
        const int ub[2] = {tri.up_base(l, 0), tri.up_base(l, 1)};
        float gf[R][NJ];  // G^{-1} as B uses it, in half the registers
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int j = 0; j < NJ; ++j) gf[r][j] = (float)gi[r][j];
        // four columns at a time: their eight entries are loaded before any
        // is rewritten (a load after a store to an offset the compiler cannot
        // tell apart would wait for its data entry by entry; only non-owned
        // entries share an offset, the sink, whose contents are never used)
        [&]<int... K>(std::integer_sequence<int, K...>) {
            auto four = [&](auto kc) __attribute__((always_inline)) {
                constexpr int j0 = 4 * decltype(kc)::value;
                int o[4][2];
                float2 cv[4][2];
                [&]<int... Q>(std::integer_sequence<int, Q...>) {
                    ((o[Q][0] = tri.template own<j0 + Q>(ub[0], l, 0, N),
                      o[Q][1] = tri.template own<j0 + Q>(ub[1], l, 1, N)), ...);
                }(std::make_integer_sequence<int, 4>{});
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int r = 0; r < 2; ++r) cv[q][r] = tri.w[o[q][r]];
                issued(cv[0][0], cv[0][1], cv[1][0], cv[1][1]);
                issued(cv[2][0], cv[2][1], cv[3][0], cv[3][1]);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
#pragma unroll
                    for (int r = 0; r < 2; ++r) {
                        const int j = j0 + q;
                        const float gv = gf[r][j];
                        const float2 v = use_evd ? make_float2(-cv[q][r].x, -cv[q][r].y)
                                                 : make_float2(gv * cv[q][r].x, gv * cv[q][r].y);
                        tri.w[o[q][r]] = v;
                        const float wgt = (o[q][r] == tri.sink()) ? 0.f : (j == l + 16 * r ? 1.f : 2.f);
                        bnorm2 = fmaf(wgt * v.x, v.x, fmaf(wgt * v.y, v.y, bnorm2));
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            };
            (four(std::integral_constant<int, K>{}), ...);
        }(std::make_integer_sequence<int, NJ / 4>{});
        wave_sync();  // B's triangle is read across lanes from here on
    }
    float mu = 0.99f;
    if (gany<64>(use_evd, 0)) {
        // EVD shift: minus a Gershgorin bound on lambda_max(C), so -C - mu I > 0
        float2 brow[R][NJ];
        if constexpr (R == 1) {
#pragma unroll
            for (int j = 0; j < NJ; ++j) brow[0][j] = lds[stid + j * kBlock];
        } else {
            tri.load(brow, true);
        }
        float rs = 0.f;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            float rsr = 0.f;
#pragma unroll
            for (int j = 0; j < NJ; ++j)
                rsr += __builtin_amdgcn_sqrtf(brow[r][j].x * brow[r][j].x + brow[r][j].y * brow[r][j].y);
            rs = fmaxf(rs, rsr);
        }
        rs = gmax<16>(rs);
        if (use_evd) mu = -(1.0f + 1e-3f) * rs - 1e-3f;
    }

    // ---- 3. shifted inverse iteration
    float2 m[R][NJ];
    bool conv;
    int it, retries;
    float2 bx[R];
    if constexpr (R == 1) {
        const BRowLds<16, NJ> bv{lds + stid, nullptr, l};
        eig_min_r<16, 1, NJ>(m, bv, bnorm2, mu, !invalid, N, l, nullptr, nullptr, nullptr, x, conv, it, retries);
        bv.apply(x, bx);
    } else {
        eig_min_r<16, R, NJ>(m, tri, bnorm2, mu, !invalid, N, l, nullptr, nullptr, nullptr, x, conv, it, retries);
        tri.apply(x, bx);
    }

    // ---- 4. eigenvalue, reference and unit phasors
    float rho = 0.f;
#pragma unroll
    for (int r = 0; r < R; ++r) rho += x[r].x * bx[r].x + x[r].y * bx[r].y;
    rho = gsum<16>(rho);
    float2 xs = x[0];
#pragma unroll
    for (int r = 1; r < R; ++r)
        if (a.ref >= 16 * r) xs = x[r];
    const int src_lane = grp * 16 + (a.ref & 15);
    const float2 xr = make_float2(__shfl(xs.x, src_lane, 64), __shfl(xs.y, src_lane, 64));
    float2 phv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = l + 16 * r;
        float2 z = make_float2(x[r].x * xr.x + x[r].y * xr.y, x[r].y * xr.x - x[r].x * xr.y);  // x conj(x_ref)
        const float z2 = z.x * z.x + z.y * z.y;
        const float zi = __builtin_amdgcn_rsqf(z2);
        phv[r] = (z2 > 0.f && !invalid) ? make_float2(z.x * zi, z.y * zi) : make_float2(1.f, 0.f);
        if (i == a.ref) phv[r] = make_float2(1.f, 0.f);
        if (live[r]) a.ph[(int64_t)i * a.ostride + pix] = phv[r];
        if (live[r] && a.phase)
            a.phase[(int64_t)i * a.ostride + pix] = (i == a.ref || invalid) ? 0.f : atan2f(phv[r].y, phv[r].x);
    }
    const uint8_t flag = invalid ? PL_FLAG_INVALID : (use_evd ? PL_FLAG_EVD : PL_FLAG_EMI);
    if (active && l == 0) {
        if (a.lam) a.lam[pix] = invalid ? __builtin_nanf("") : (use_evd ? -rho : rho);
        if (a.flags) a.flags[pix] = flag;
    }
    if (a.tcoh) {
        // ---- 5. temporal coherence: row i contributes
        // conj(zeta_i) sum_{k > i} u(C_ik) zeta_k; zeta_k comes from lane k % 16
        // (slot k / 16) by DPP broadcast, in uniform control flow
        const float2* mat3 = mat + opaque_int(0);
        float sre = 0.f, sim = 0.f;
        [&]<int... K>(std::integer_sequence<int, K...>) {
            float2 acc[R];
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = make_float2(0.f, 0.f);
            auto one = [&](auto kc) __attribute__((always_inline)) {
                constexpr int k = decltype(kc)::value;
                const float zx = rowcast<k % 16>(phv[k / 16].x), zy = rowcast<k % 16>(phv[k / 16].y);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int i = l + 16 * r;
                    const bool use = live[r] && k > i && k < N;
                    const float2 cv = mat3[centry(packed, N, min(i, N - 1), min(k, N - 1))];
                    const float c2 = cv.x * cv.x + cv.y * cv.y;
                    const float q = __builtin_amdgcn_rsqf(c2);
                    const float2 u = c2 > 0.f ? make_float2(cv.x * q, cv.y * q) : make_float2(1.f, 0.f);
                    acc[r].x += use ? u.x * zx - u.y * zy : 0.f;
                    acc[r].y += use ? u.x * zy + u.y * zx : 0.f;
                }
            };
            (one(std::integral_constant<int, K>{}), ...);
#pragma unroll
            for (int r = 0; r < R; ++r) {  // conj(zeta_i) acc
                sre += phv[r].x * acc[r].x + phv[r].y * acc[r].y;
                sim += phv[r].x * acc[r].y - phv[r].y * acc[r].x;
            }
        }(std::make_integer_sequence<int, NJ>{});
        sre = gsum<16>(sre);
        sim = gsum<16>(sim);
        const float nifg = 0.5f * (float)N * (float)(N - 1);
        float gt = N > 1 ? __builtin_sqrtf(sre * sre + sim * sim) / nifg : 1.f;
        if (invalid) gt = 0.f;
        if (active && l == 0) a.tcoh[pix] = gt;
    }
    if (a.counters) {
        const bool lead = active && l == 0;
        const uint64_t e = __ballot(lead && flag == PL_FLAG_EVD);
        const uint64_t v = __ballot(lead && flag == PL_FLAG_INVALID);
        const uint64_t nc = __ballot(lead && !conv);
        const int rt = (int)gsum<64>(lead ? (float)retries : 0.f);
        const int its = (int)gsum<64>(lead ? (float)it : 0.f);
        if (lane == 0) {
            if (e) atomicAdd(a.counters + PL_CNT_EVD, (unsigned long long)__popcll(e));
            if (v) atomicAdd(a.counters + PL_CNT_INVALID, (unsigned long long)__popcll(v));
            if (nc) atomicAdd(a.counters + PL_CNT_NOT_CONVERGED, (unsigned long long)__popcll(nc));
            if (rt) atomicAdd(a.counters + PL_CNT_SHIFT_RETRY, (unsigned long long)rt);
            if (its) atomicAdd(a.counters + PL_CNT_ITERS, (unsigned long long)its);
        }
        // histogram of iterations per pixel (bin 15: 15 or more)
        const int bin = it < 15 ? it : 15;
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            const uint64_t hb = __ballot(lead && !invalid && bin == b);
            if (lane == 0 && hb) atomicAdd(a.counters + PL_CNT_ITER_HIST + b, (unsigned long long)__popcll(hb));
        }
    }
}

}  // namespace
}  // namespace plk
