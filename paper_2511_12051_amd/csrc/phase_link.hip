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
#include "link_device.hpp"

namespace plk {
namespace {

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
    __shared__ __attribute__((aligned(16))) float2 lds[link_lds_bytes<R, NJ>() / 8];
    if constexpr (R == 1) {
        link_body<R, NJ>(a, blockIdx.x, threadIdx.x, lds);
    } else {
        for (int64_t b = blockIdx.x; b < blocks; b += gridDim.x) link_body<R, NJ>(a, b, threadIdx.x, lds);
    }
}

// the stride loop needs more registers: allow occupancy 3 for one-row groups
// rather than spilling
template <int R, int NJ>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(R == 1 ? 3 : 2, R == 1 ? 4 : 2)))
void phase_link_batch(BatchRange<LinkArgs> r) {
    // groups of a block never synchronise with each other, so consecutive
    // blocks of the stride loop need no barrier
    __shared__ __attribute__((aligned(16))) float2 lds[link_lds_bytes<R, NJ>() / 8];
    for (int64_t b = blockIdx.x; b < r.total; b += gridDim.x) {
        const int k = batch_item(r.starts, r.n, b);
        link_body<R, NJ>(r.items[k], b - r.starts[k], threadIdx.x, lds);
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
