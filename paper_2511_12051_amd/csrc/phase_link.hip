// EMI phase linking with EVD fallback (paper Sec. 3.2, eq.
// emi-eigenvalue-problem) and the reference gauge of Sec. 2.1.
//
// Layout: a group of 16 lanes (one DPP row) owns one pixel and lane l holds
// rows l and, for N > 16, l + 16 of every matrix in registers (N <= 32
// images), so a wavefront solves 4 pixels side by side.  The pivot row of
// each Gauss-Jordan step and the current iterate move between the lanes of a
// group by DPP row broadcasts; B is kept in LDS between factorisations.
//
//  1. G = |C| in FP64; in-place Gauss-Jordan inversion.  Its pivots are the
//     LDL^T pivots of G; one <= 1e-6 (or not finite) means the inversion
//     failed and the pixel takes the EVD branch.
//  2. B = G^{-1} o C (EMI) or B = -C (EVD); both need the eigenvector of the
//     smallest eigenvalue of the Hermitian B.
//  3. Shifted inverse iteration with an explicit (B - mu I)^{-1} in FP32,
//     formed by complex Gauss-Jordan on the vector ALUs for N <= 16 and, for
//     N > 16, by a Hermitian sweep on the matrix cores, one pixel's matrix
//     per 32 x 32 accumulator pair (each step a complex rank-1 update, two
//     v_mfma_f32_32x32x2f32).  All pivots positive proves
//     mu < lambda_min (Sylvester's inertia), so the iteration converges to the
//     wanted eigenvector.  EMI starts from mu = 0.99 (Sec. 3.2) and backs off
//     if the inertia check fails; EVD starts from minus the largest absolute
//     row sum of C (a Gershgorin bound).  When the iterate contracts slowly
//     (checked after 4, 8, 12 and 18 steps) the shift moves up to
//     rho - f ||B x - rho x|| (rho the Rayleigh quotient, f = 1, 2, 4 until
//     the inertia check accepts one); this keeps the iteration count low when
//     the eigen-gap is small compared with the distance from 0.99.
//  4. zeta_i = x_i conj(x_ref), returned as unit phasors.
//  5. Optionally the temporal coherence of the result (Sec. 3.3,
//     eq. temporal-coherence): gamma_t = |sum_{i<k} u(C_ik) conj(zeta_i)
//     zeta_k| / (N(N-1)/2), u(c) = c / |c| (1 for c = 0), from C's upper
//     triangle re-read from cache and zeta broadcast between the lanes.
//
// C arrives either as full matrices or as packed upper triangles (row-major
// entries (i, j >= i)); with the packed layout every row reads the Hermitian
// matrix of the upper triangle.
#include <cmath>
#include <utility>

#include "batch_device.hpp"
#include "eig_device.hpp"

namespace plk {
namespace {

// offset of entry (i, j), i <= j, inside one pixel's matrix
__device__ __forceinline__ int centry(int packed, int N, int i, int j) {
    return packed ? ((i * (2 * N - i - 1)) >> 1) + j : i * N + j;
}

template <int R, int NJ>
__device__ __forceinline__ void link_body(const LinkArgs& a, int64_t block) {
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
    constexpr int LDS_BYTES = R == 1 ? NJ * kBlock * 8 : (kBlock / 64) * (Tri::WAVE_ENTRIES + XS) * 8;
    __shared__ __attribute__((aligned(16))) float2 lds[LDS_BYTES / 8];
    // opaque copies of the lane index and N: in a persistent loop the
    // compiler would otherwise precompute every per-step constant and
    // predicate once and keep them live (in spilled registers) across it
    const int lane = opaque_int(lane_id());
    const int l = lane & 15;
    const int grp = lane >> 4;
    const int wave = threadIdx.x >> 6;

    const int N = opaque_uniform(__builtin_amdgcn_readfirstlane(a.N));
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
    const Tri tri{lds + wave * Tri::WAVE_ENTRIES, grp, l, N, lds + (kBlock / 64) * Tri::WAVE_ENTRIES + wave * XS};
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
        for (int j = 0; j < NJ; ++j) gi[r][j] = (live[r] && j < N) ? cabs64(c[r][j].x, c[r][j].y) : 0.0;
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
        float2* bme = lds + threadIdx.x;  // element j at bme[j * kBlock]
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
        [&]<int... J>(std::integer_sequence<int, J...>) {
            auto one = [&](auto jc, int r) __attribute__((always_inline)) {
                constexpr int j = decltype(jc)::value;
                const int o = tri.template own<j>(ub[r], l, r, N);
                const float2 cv = tri.w[o];
                const float gv = gf[r][j];
                const float2 v = use_evd ? make_float2(-cv.x, -cv.y) : make_float2(gv * cv.x, gv * cv.y);
                tri.w[o] = v;
                const float wgt = (o == tri.sink()) ? 0.f : (j == l + 16 * r ? 1.f : 2.f);
                bnorm2 = fmaf(wgt * v.x, v.x, fmaf(wgt * v.y, v.y, bnorm2));
            };
            // at most four columns of loads in flight
            auto four = [&](auto jc) __attribute__((always_inline)) {
                constexpr int j = decltype(jc)::value;
#pragma unroll
                for (int r = 0; r < R; ++r) one(jc, r);
                if constexpr (j % 4 == 3) __builtin_amdgcn_sched_barrier(0);
            };
            (four(std::integral_constant<int, J>{}), ...);
        }(std::make_integer_sequence<int, NJ>{});
        wave_sync();  // B's triangle is read across lanes from here on
    }
    float mu = 0.99f;
    if (gany<64>(use_evd, 0)) {
        // EVD shift: minus a Gershgorin bound on lambda_max(C), so -C - mu I > 0
        float2 brow[R][NJ];
        if constexpr (R == 1) {
#pragma unroll
            for (int j = 0; j < NJ; ++j) brow[0][j] = lds[threadIdx.x + j * kBlock];
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
        const BRowLds<16, NJ> bv{lds + threadIdx.x, nullptr, l};
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

// Groups with two rows per lane (N > 16) run persistently: the grid (16
// times the resident workgroups) strides over the pixel blocks, which avoids
// dispatching hundreds of thousands of short workgroups; one-row groups keep
// one block per workgroup.  Two-row kernels are held to two wavefronts per
// SIMD: within 256 registers a few dozen values spill, all outside the
// solver loop, and that measured 28 % faster at 28 columns than one
// wavefront per SIMD without spills.
template <int R, int NJ>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(R == 1 ? 4 : 2, R == 1 ? 4 : 2)))
void phase_link_kernel(LinkArgs a, int64_t blocks) {
    if constexpr (R == 1) {
        link_body<R, NJ>(a, blockIdx.x);
    } else {
        for (int64_t b = blockIdx.x; b < blocks; b += gridDim.x) link_body<R, NJ>(a, b);
    }
}

// the stride loop needs more registers: allow occupancy 3 for one-row groups
// rather than spilling
template <int R, int NJ>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(R == 1 ? 3 : 2, R == 1 ? 4 : 2)))
void phase_link_batch(BatchRange<LinkArgs> r) {
    // groups of a block never synchronise with each other, so consecutive
    // blocks of the stride loop need no barrier
    for (int64_t b = blockIdx.x; b < r.total; b += gridDim.x) {
        const int k = batch_item(r.starts, r.n, b);
        link_body<R, NJ>(r.items[k], b - r.starts[k]);
    }
}

}  // namespace

int64_t link_blocks(int N, int64_t npix) {
    (void)N;
    const int64_t per_block = (kBlock / 64) * 4;  // four 16-lane groups per wavefront
    return (npix + per_block - 1) / per_block;
}

template <int R, int NJ>
pl_status launch_persistent(const LinkArgs& a, int64_t blocks, hipStream_t s) {
    // resident workgroups per CU of this variant, per device (queried once)
    static int per_cu[64] = {0};
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (!per_cu[dev]) {
        int n = 0, c = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(phase_link_kernel<R, NJ>),
                                                         kBlock, 0) != hipSuccess || n < 1)
            n = 1;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1) c = 1;
        cus[dev] = c;
        per_cu[dev] = n;
    }
    int64_t grid = R == 1 ? blocks : (int64_t)per_cu[dev] * cus[dev] * 16;  // 16: measured best of 2, 4, 8, 16
    if (grid > blocks) grid = blocks;
    if (grid > 2147483647LL) return fail(PL_ERR_UNSUPPORTED, "pl_phase_link: too many pixels");
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL((phase_link_kernel<R, NJ>), dim3((unsigned)grid), dim3(kBlock), 0, s, a, blocks);
    return launch_ok("phase linking kernel");
}

LinkArgs link_args(const float2* coh, int N, int64_t npix, int ref, int method, float2* phasors,
                   float* phase, float* lambda, uint8_t* flags, unsigned long long* counters) {
    LinkArgs a{coh, N, npix, ref, method, phasors, phase, lambda, flags, counters, nullptr, 0, npix};
    return a;
}

pl_status launch_phase_link(const LinkArgs& a, hipStream_t s) {
    const int64_t blocks = link_blocks(a.N, a.npix);
    switch ((a.N + 3) / 4) {  // columns per row: N rounded up to a multiple of 4
        case 1: case 2: case 3: return launch_persistent<1, 12>(a, blocks, s);
        case 4: return launch_persistent<1, 16>(a, blocks, s);
        case 5: return launch_persistent<2, 20>(a, blocks, s);
        case 6: return launch_persistent<2, 24>(a, blocks, s);
        case 7: return launch_persistent<2, 28>(a, blocks, s);
        default: return launch_persistent<2, 32>(a, blocks, s);
    }
}

const void* phase_link_batch_fn(int N_class) {
    switch (N_class) {
        case 1: case 2: case 3: return reinterpret_cast<const void*>(phase_link_batch<1, 12>);
        case 4: return reinterpret_cast<const void*>(phase_link_batch<1, 16>);
        case 5: return reinterpret_cast<const void*>(phase_link_batch<2, 20>);
        case 6: return reinterpret_cast<const void*>(phase_link_batch<2, 24>);
        case 7: return reinterpret_cast<const void*>(phase_link_batch<2, 28>);
        default: return reinterpret_cast<const void*>(phase_link_batch<2, 32>);
    }
}

pl_status launch_phase_link_batch(const BatchRange<LinkArgs>& r, int N_class, int64_t grid, hipStream_t s) {
    if (r.total == 0) return PL_OK;
    const dim3 gr((unsigned)grid), block(kBlock);
    switch (N_class) {  // (N + 3) / 4, shared by every item of the range
        case 1: case 2: case 3: hipLaunchKernelGGL((phase_link_batch<1, 12>), gr, block, 0, s, r); break;
        case 4: hipLaunchKernelGGL((phase_link_batch<1, 16>), gr, block, 0, s, r); break;
        case 5: hipLaunchKernelGGL((phase_link_batch<2, 20>), gr, block, 0, s, r); break;
        case 6: hipLaunchKernelGGL((phase_link_batch<2, 24>), gr, block, 0, s, r); break;
        case 7: hipLaunchKernelGGL((phase_link_batch<2, 28>), gr, block, 0, s, r); break;
        default: hipLaunchKernelGGL((phase_link_batch<2, 32>), gr, block, 0, s, r); break;
    }
    return launch_ok("batched phase linking kernel");
}

}  // namespace plk
