// EMI phase linking with EVD fallback (paper Sec. 3.2, eq.
// emi-eigenvalue-problem) and the reference gauge of Sec. 2.1.
//
// Layout: a group of NP = 16 or 32 lanes owns one pixel, lane i holds row i of
// every matrix in registers (NP <= 32 images), so a wavefront solves 4 or 2
// pixels side by side.  The pivot row of each Gauss-Jordan step and the
// current iterate are broadcast through a few hundred bytes of LDS per group.
//
//  1. G = |C| in FP64; in-place Gauss-Jordan inversion.  Its pivots are the
//     LDL^T pivots of G; one <= 1e-6 (or not finite) means the inversion
//     failed and the pixel takes the EVD branch.
//  2. B = G^{-1} o C (EMI) or B = -C (EVD); both need the eigenvector of the
//     smallest eigenvalue of the Hermitian B.
//  3. Shifted inverse iteration with an explicit (B - mu I)^{-1}, formed by
//     complex Gauss-Jordan in FP32.  All pivots positive proves
//     mu < lambda_min (Sylvester's inertia), so the iteration converges to the
//     wanted eigenvector.  EMI starts from mu = 0.99 (Sec. 3.2) and backs off
//     if the inertia check fails; EVD starts from minus the largest absolute
//     row sum of C (a Gershgorin bound).  When the iterate contracts slowly
//     (checked after 4, 8, 12 and 18 steps) the shift moves up to
//     rho - f ||B x - rho x|| (rho the Rayleigh quotient, f = 1, 2, 4 until
//     the inertia check accepts one); this keeps the iteration count low when
//     the eigen-gap is small compared with the distance from 0.99.
//  4. zeta_i = x_i conj(x_ref), returned as unit phasors.
#include <cmath>

#include "batch_device.hpp"
#include "eig_device.hpp"

namespace plk {
namespace {



template <int NP, int NJ>
__device__ __forceinline__ void link_body(const LinkArgs& a, int64_t block) {
    constexpr int GPW = 64 / NP;  // groups (pixels) per wavefront
    // NJ >= N columns are stored and updated per row (N rounded up to a
    // multiple of 4); NP >= N lanes hold the rows.
    // per group: two GJ pivot-row buffers (NJ + 2 doubles each, also used as
    // NJ + 2 float2) and the iterate buffer (NP float2)
    constexpr int ROW_BYTES = (NJ + 2) * 8;
    constexpr int GROUP_BYTES = 2 * ROW_BYTES + NP * 8;
    __shared__ __attribute__((aligned(16))) unsigned char lds[(kBlock / 64) * GPW * GROUP_BYTES];
    // row i of B for every lane, element-major so that the lanes of a
    // wavefront read consecutive words: read back for refactorisations and
    // Rayleigh quotients instead of occupying registers through the iteration
    __shared__ __attribute__((aligned(16))) float2 brow[NJ][kBlock];
    const int lane = lane_id();
    const int i = lane & (NP - 1);
    const int grp = lane / NP;
    const int wave = threadIdx.x >> 6;
    unsigned char* gbase = lds + (wave * GPW + grp) * GROUP_BYTES;
    double* rbd0 = reinterpret_cast<double*>(gbase);
    double* rbd1 = reinterpret_cast<double*>(gbase + ROW_BYTES);
    float2* rbc0 = reinterpret_cast<float2*>(gbase);
    float2* rbc1 = reinterpret_cast<float2*>(gbase + ROW_BYTES);
    float2* xb = reinterpret_cast<float2*>(gbase + 2 * ROW_BYTES);

    const int N = a.N;
    const int64_t pix = (block * (kBlock / 64) + wave) * GPW + grp;
    const bool active = pix < a.npix;
    const bool row_live = active && i < N;

    // ---- row i of C (each lane reads its own row; a variant staging the
    // wavefront's matrices through LDS with coalesced loads measured slower)
    const int NN = N * N;
    const float2* src = a.coh + (active ? pix : 0) * (int64_t)NN + (int64_t)i * N;
    float2 c[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) c[j] = (row_live && j < N) ? src[j] : make_float2(0.f, 0.f);
    bool bad = false;
#pragma unroll
    for (int j = 0; j < NJ; ++j) bad = bad || !(fabsf(c[j].x) <= 3.4e38f && fabsf(c[j].y) <= 3.4e38f);
    const bool invalid = !active || gany<NP>(bad, grp);

    // start from column ref of C: the single-reference interferogram phases
    float2 x = make_float2(0.f, 0.f);
#pragma unroll
    for (int j = 0; j < NJ; ++j)
        if (j == a.ref && row_live) x = c[j];
    {
        // unit-modulus start: the phases of column ref (for consistent phases
        // the EMI eigenvector has entries of equal modulus)
        const float x2 = x.x * x.x + x.y * x.y;
        if (x2 > 0.f) {
            const float r = __builtin_amdgcn_rsqf(x2);
            x.x *= r;
            x.y *= r;
        }
        float nrm = gsum<NP>(x.x * x.x + x.y * x.y);
        if (!(nrm > 0.f)) {
            x = make_float2(i == a.ref ? 1.f : 0.f, 0.f);
            nrm = 1.f;
        }
        const float s = __builtin_amdgcn_rsqf(nrm);
        x.x *= s;
        x.y *= s;
    }
    // ---- 1. FP64 inverse of G = |C|
    bool use_evd = a.method == PL_LINK_EVD;
    double gi[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) gi[j] = (row_live && j < N) ? cabs64(c[j].x, c[j].y) : 0.0;
    const bool do_emi = !use_evd && !invalid;
    const bool gfail = factor_g<NP, NJ>(gi, N, i, do_emi, rbd0, rbd1);
    use_evd = use_evd || gfail;

    // ---- 2. the Hermitian matrix whose smallest eigenpair is wanted.  Row i
    // of C is read again (an L2 hit) rather than kept live across step 1.
#pragma unroll
    for (int j = 0; j < NJ; ++j) c[j] = (row_live && j < N) ? src[j] : make_float2(0.f, 0.f);
    float2* bme = &brow[0][threadIdx.x];  // element j at bme[j * kBlock]
    float bnorm2 = 0.f;  // ||row i of B||^2
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        float2 v;
        if (use_evd) v = make_float2(-c[j].x, -c[j].y);
        else v = make_float2((float)gi[j] * c[j].x, (float)gi[j] * c[j].y);
        bme[j * kBlock] = v;
        bnorm2 += v.x * v.x + v.y * v.y;
    }
    float mu = 0.99f;
    if (use_evd) {
        // EVD shift: minus a Gershgorin bound on lambda_max(C), so -C - mu I > 0
        float rs = 0.f;
#pragma unroll
        for (int j = 0; j < NJ; ++j) rs += __builtin_amdgcn_sqrtf(c[j].x * c[j].x + c[j].y * c[j].y);
        mu = -(1.0f + 1e-3f) * gmax<NP>(rs) - 1e-3f;
    }

    // ---- 3. shifted inverse iteration
    float2 m[NJ];
    bool conv;
    int it, retries;
    eig_min<NP, NJ>(m, bme, bnorm2, mu, !invalid, N, i, rbc0, rbc1, xb, x, conv, it, retries);

    // ---- 4. eigenvalue, reference and unit phasors
    const float2 bx = group_matvec_lds<NP, NJ>(bme, x, i, xb);
    const float rho = gsum<NP>(x.x * bx.x + x.y * bx.y);
    const float2 xr = make_float2(__shfl(x.x, grp * NP + a.ref, 64), __shfl(x.y, grp * NP + a.ref, 64));
    float2 z = make_float2(x.x * xr.x + x.y * xr.y, x.y * xr.x - x.x * xr.y);  // x conj(x_ref)
    const float z2 = z.x * z.x + z.y * z.y;
    const float zi = __builtin_amdgcn_rsqf(z2);
    float2 phv = (z2 > 0.f && !invalid) ? make_float2(z.x * zi, z.y * zi) : make_float2(1.f, 0.f);
    if (i == a.ref) phv = make_float2(1.f, 0.f);
    if (row_live) a.ph[(int64_t)i * a.npix + pix] = phv;
    if (row_live && a.phase) a.phase[(int64_t)i * a.npix + pix] = (i == a.ref || invalid) ? 0.f : atan2f(phv.y, phv.x);
    const uint8_t flag = invalid ? PL_FLAG_INVALID : (use_evd ? PL_FLAG_EVD : PL_FLAG_EMI);
    if (active && i == 0) {
        if (a.lam) a.lam[pix] = invalid ? __builtin_nanf("") : (use_evd ? -rho : rho);
        if (a.flags) a.flags[pix] = flag;
    }
    if (a.counters) {
        const bool lead = active && i == 0;
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
    }
}

// 32-lane groups (N > 16) run persistently: the grid (a few times the
// resident workgroups) strides over the pixel blocks, which avoids
// dispatching hundreds of thousands of short workgroups; 16-lane groups keep
// one block per workgroup, where the loop would cost the occupancy-4
// register budget
template <int NP, int NJ>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(NP == 16 ? 4 : 1, NP == 16 ? 4 : 2)))
void phase_link_kernel(LinkArgs a, int64_t blocks) {
    if constexpr (NP == 16) {
        link_body<NP, NJ>(a, blockIdx.x);
    } else {
        for (int64_t b = blockIdx.x; b < blocks; b += gridDim.x) link_body<NP, NJ>(a, b);
    }
}

// the stride loop needs a few registers more than 128: allow occupancy 3 for
// 16-lane groups rather than spilling
template <int NP, int NJ>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(NP == 16 ? 3 : 1, NP == 16 ? 4 : 2)))
void phase_link_batch(BatchRange<LinkArgs> r) {
    // groups of a block never synchronise with each other, so consecutive
    // blocks of the stride loop need no barrier
    for (int64_t b = blockIdx.x; b < r.total; b += gridDim.x) {
        const int k = batch_item(r.starts, r.n, b);
        link_body<NP, NJ>(r.items[k], b - r.starts[k]);
    }
}

}  // namespace

int64_t link_blocks(int N, int64_t npix) {
    const int np = N <= 16 ? 16 : 32;
    const int64_t per_block = (kBlock / 64) * (64 / np);
    return (npix + per_block - 1) / per_block;
}

template <int NP, int NJ>
pl_status launch_persistent(const LinkArgs& a, int64_t blocks, hipStream_t s) {
    // resident workgroups per CU of this variant, per device (queried once)
    static int per_cu[64] = {0};
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (!per_cu[dev]) {
        int n = 0, c = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(phase_link_kernel<NP, NJ>),
                                                         kBlock, 0) != hipSuccess || n < 1)
            n = 1;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1) c = 1;
        cus[dev] = c;
        per_cu[dev] = n;
    }
    int64_t grid = NP == 16 ? blocks : (int64_t)per_cu[dev] * cus[dev] * 4;
    if (grid > blocks) grid = blocks;
    if (grid > 2147483647LL) return fail(PL_ERR_UNSUPPORTED, "pl_phase_link: too many pixels");
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL((phase_link_kernel<NP, NJ>), dim3((unsigned)grid), dim3(kBlock), 0, s, a, blocks);
    return launch_ok("phase linking kernel");
}

pl_status launch_phase_link(const float2* coh, int N, int64_t npix, int ref, int method,
                            float2* phasors, float* phase, float* lambda, uint8_t* flags,
                            unsigned long long* counters, hipStream_t s) {
    LinkArgs a{coh, N, npix, ref, method, phasors, phase, lambda, flags, counters};
    const int64_t blocks = link_blocks(N, npix);
    switch ((N + 3) / 4) {  // columns per row: N rounded up to a multiple of 4
        case 1: case 2: case 3: return launch_persistent<16, 12>(a, blocks, s);
        case 4: return launch_persistent<16, 16>(a, blocks, s);
        case 5: return launch_persistent<32, 20>(a, blocks, s);
        case 6: return launch_persistent<32, 24>(a, blocks, s);
        case 7: return launch_persistent<32, 28>(a, blocks, s);
        default: return launch_persistent<32, 32>(a, blocks, s);
    }
}

const void* phase_link_batch_fn(int N_class) {
    switch (N_class) {
        case 1: case 2: case 3: return reinterpret_cast<const void*>(phase_link_batch<16, 12>);
        case 4: return reinterpret_cast<const void*>(phase_link_batch<16, 16>);
        case 5: return reinterpret_cast<const void*>(phase_link_batch<32, 20>);
        case 6: return reinterpret_cast<const void*>(phase_link_batch<32, 24>);
        case 7: return reinterpret_cast<const void*>(phase_link_batch<32, 28>);
        default: return reinterpret_cast<const void*>(phase_link_batch<32, 32>);
    }
}

pl_status launch_phase_link_batch(const BatchRange<LinkArgs>& r, int N_class, int64_t grid, hipStream_t s) {
    if (r.total == 0) return PL_OK;
    const dim3 gr((unsigned)grid), block(kBlock);
    switch (N_class) {  // (N + 3) / 4, shared by every item of the range
        case 1: case 2: case 3: hipLaunchKernelGGL((phase_link_batch<16, 12>), gr, block, 0, s, r); break;
        case 4: hipLaunchKernelGGL((phase_link_batch<16, 16>), gr, block, 0, s, r); break;
        case 5: hipLaunchKernelGGL((phase_link_batch<32, 20>), gr, block, 0, s, r); break;
        case 6: hipLaunchKernelGGL((phase_link_batch<32, 24>), gr, block, 0, s, r); break;
        case 7: hipLaunchKernelGGL((phase_link_batch<32, 28>), gr, block, 0, s, r); break;
        default: hipLaunchKernelGGL((phase_link_batch<32, 32>), gr, block, 0, s, r); break;
    }
    return launch_ok("batched phase linking kernel");
}

}  // namespace plk
