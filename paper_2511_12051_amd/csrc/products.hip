// Products built on the linked phases:
//  - persistent-scatterer selection by the amplitude dispersion
//    D_A = sigma_A / mu_A (paper Sec. 3.1, threshold of Sec. 4) and the
//    regridding of PS and DS phases to the output grid (supplement,
//    "Regridding PS and DS to 30 m resolution");
//  - the phase cosine similarity gamma_s (Sec. 3.3, eq. phase-cosine-sim)
//    over the nearest-k interferogram network (Sec. 3.4);
//  - the L1 network inversion of unwrapped interferograms (Sec. 3.5,
//    eq. l1-min) by the ADMM iteration of Appendix A.
// (The temporal coherence gamma_t is an epilogue of the linking kernel.)
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace plk {
namespace {

constexpr int kBlock = 256;

// ------------------------------------------------------------ PS regridding
// One thread per output pixel scans its block, the full-resolution pixels that
// map to it (rows min(y / sy, oR - 1) == by, likewise for columns, so the
// last block also takes the ragged edge), in row-major order.  D_A is formed
// in FP64 from the FP64 statistics; the first PS of lowest D_A wins.
struct RegridArgs {
    PlaneTable t;
    int N, ref;
    Geometry g;
    const double* mean;
    const double* var;
    double thr;
    const float2* ds;   // [N][P]
    float2* out;        // [N][P] (may alias ds)
    int64_t* src;       // [P] or null
    uint8_t* ps;        // [R][C] or null
};

__global__ __launch_bounds__(kBlock) void ps_regrid_kernel(RegridArgs a) {
    const Geometry& g = a.g;
    const int64_t P = g.oR * g.oC;
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= P) return;
    const int64_t by = p / g.oC, bx = p - by * g.oC;
    const int64_t y0 = by * g.sy, y1 = by + 1 == g.oR ? g.R : y0 + g.sy;
    const int64_t x0 = bx * g.sx, x1 = bx + 1 == g.oC ? g.C : x0 + g.sx;
    double best = INFINITY;
    int64_t q = -1;
    for (int64_t y = y0; y < y1; ++y) {
        for (int64_t x = x0; x < x1; ++x) {
            const int64_t k = y * g.C + x;
            const double mu = a.mean[k];
            const double da = sqrt(fmax(a.var[k], 0.0)) / mu;
            const bool is_ps = mu > 0.0 && da <= a.thr;  // false for NaN / inf
            if (a.ps) a.ps[k] = is_ps ? 1 : 0;
            if (is_ps && da < best) {
                best = da;
                q = k;
            }
        }
    }
    if (a.src) a.src[p] = q;
    if (q < 0) {
        if (a.out != a.ds)
            for (int i = 0; i < a.N; ++i) a.out[(int64_t)i * P + p] = a.ds[(int64_t)i * P + p];
        return;
    }
    const float2 zr = a.t.p[a.ref][q];
    for (int i = 0; i < a.N; ++i) {
        const float2 zi = a.t.p[i][q];
        // z_i conj(z_ref) as a unit phasor (angle 0 where it vanishes)
        const float re = zi.x * zr.x + zi.y * zr.y, im = zi.y * zr.x - zi.x * zr.y;
        const float n2 = re * re + im * im;
        const float s = __builtin_amdgcn_rsqf(n2);
        float2 v = n2 > 0.f && n2 <= 3.4e38f ? make_float2(re * s, im * s) : make_float2(1.f, 0.f);
        if (i == a.ref) v = make_float2(1.f, 0.f);
        a.out[(int64_t)i * P + p] = v;
    }
}

// ------------------------------------------------------- phase similarity
// One wavefront per output pixel p.  Lane l takes the positions
// s = l + 64 t of the (2r+1)^2 square around p (t < 16, so r <= 15) and keeps
// those inside the disk, the grid and not flagged invalid, the centre
// excluded.  For a neighbour q, with u_a = zeta_a(p) conj(zeta_a(q)):
//   s(p, q) = (1/N_ifg) sum_{1 <= b - a <= k} Re(u_a conj(u_b))
//           = mean over the network of cos((phi_a - phi_b)(p) - (phi_a - phi_b)(q)).
// gamma_s is the median of the kept values (mean of the two middle ones for
// an even count), found by two radix selections on order-preserving keys.
constexpr int kSimSlots = 16;

struct SimArgs {
    const float2* ph;  // [N][P]
    const uint8_t* flags;
    int64_t oR, oC;
    int N, k, radius;
    float* out;
};

__device__ __forceinline__ uint32_t order_key(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key_value(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// k-th smallest (0-based) of the kept keys of the wavefront
__device__ uint32_t wave_select(const uint32_t (&key)[kSimSlots], const bool (&keep)[kSimSlots], int k) {
    uint32_t prefix = 0;
    for (int bit = 31; bit >= 0; --bit) {
        const uint32_t want = prefix >> bit;  // bits above `bit` as chosen, this bit 0
        int c = 0;
#pragma unroll
        for (int t = 0; t < kSimSlots; ++t) c += (keep[t] && (key[t] >> bit) == want) ? 1 : 0;
        c = wave_sum_int(c);
        if (k >= c) {
            k -= c;
            prefix |= 1u << bit;
        }
    }
    return prefix;
}

__global__ __launch_bounds__(kBlock) void phase_similarity_kernel(SimArgs a) {
    __shared__ float2 zp_all[kBlock / 64][kMaxN];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t P = a.oR * a.oC;
    const int64_t p = (int64_t)blockIdx.x * (kBlock / 64) + wave;
    if (p >= P) return;  // uniform per wavefront
    const int N = a.N;
    float2* zp = zp_all[wave];
    if (lane < N) zp[lane] = a.ph[(int64_t)lane * P + p];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const bool p_ok = !(a.flags && a.flags[p] == PL_FLAG_INVALID);
    const int64_t py = p / a.oC, px = p - py * a.oC;
    const int r = a.radius, side = 2 * r + 1;
    int nifg = 0;
    for (int d = 1; d <= a.k; ++d) nifg += N - d > 0 ? N - d : 0;
    const float inv_nifg = nifg > 0 ? 1.f / (float)nifg : 0.f;
    uint32_t key[kSimSlots];
    bool keep[kSimSlots];
#pragma unroll
    for (int t = 0; t < kSimSlots; ++t) {
        const int s = lane + 64 * t;
        const int dy = s / side - r, dx = s % side - r;
        const int64_t qy = py + dy, qx = px + dx;
        bool use = s < side * side && (dy | dx) != 0 && dy * dy + dx * dx <= r * r && qy >= 0 && qy < a.oR &&
                   qx >= 0 && qx < a.oC;
        const int64_t q = use ? qy * a.oC + qx : p;
        if (use && a.flags && a.flags[q] == PL_FLAG_INVALID) use = false;
        float acc = 0.f;
        if (use && nifg > 0) {
            float2 u1 = make_float2(0.f, 0.f), u2 = u1, u3 = u1;  // u_{a-1}, u_{a-2}, u_{a-3}
            for (int i = 0; i < N; ++i) {
                const float2 zq = a.ph[(int64_t)i * P + q];
                const float2 z = zp[i];
                const float2 u = make_float2(z.x * zq.x + z.y * zq.y, z.y * zq.x - z.x * zq.y);  // z conj(zq)
                // Re(u_{i-d} conj(u_i)) for the pairs (i - d, i), d = 1..k
                if (i >= 1 && a.k >= 1) acc += u1.x * u.x + u1.y * u.y;
                if (i >= 2 && a.k >= 2) acc += u2.x * u.x + u2.y * u.y;
                if (i >= 3 && a.k >= 3) acc += u3.x * u.x + u3.y * u.y;
                u3 = u2;
                u2 = u1;
                u1 = u;
            }
        }
        keep[t] = use;
        key[t] = order_key(nifg > 0 ? acc * inv_nifg : 1.f);
    }
    int n = 0;
#pragma unroll
    for (int t = 0; t < kSimSlots; ++t) n += keep[t] ? 1 : 0;
    n = wave_sum_int(n);
    float med = 0.f;
    if (p_ok && n > 0) {
        const float hi = key_value(wave_select(key, keep, n / 2));
        med = (n & 1) ? hi : 0.5f * (key_value(wave_select(key, keep, n / 2 - 1)) + hi);
    }
    if (lane == 0) a.out[p] = med;
}

// ------------------------------------------------------- ADMM L1 inversion
// One thread per pixel.  Interferogram j of the nearest-k network is the pair
// (a, a + d) with separation d = 1..k, numbered by d, then a (the order of
// the input rows); x_c is the phase of date c + 1 relative to date 0.  Per
// iteration (Appendix A, z^0 = u^0 = 0):
//   x = (A^T A)^{-1} A^T (b + z - u)    banded Cholesky solve (bandwidth k)
//   t = A x - b + u,  z = S_{1/rho}(t),  u = t - z.
// The factor of A^T A is shared by all pixels and arrives in the arguments:
// its diagonal's reciprocals and k sub-diagonals, identity beyond date N - 1,
// so that a kernel sized for NX dates runs any N <= NX + 1.  Up to 16 dates
// the interferograms stay in registers (BREG); above, they are read again
// from cache in every iteration, which keeps z and u in registers.
constexpr int kNet = 3;

struct AdmmArgs {
    const float* b;    // [n_ifg][P]
    float* x;          // [N - 1][P]
    float* resid;      // [P] sum |A x - b| at the end, or null
    int64_t P;
    int N, k, iters;
    float kappa;       // 1 / rho
    float inv_diag[kMaxN];
    float sub[kNet][kMaxN];  // sub[d-1][c] = L[c][c - d]
};

template <int NX, bool BREG>
__global__ __launch_bounds__(kBlock) void admm_kernel(AdmmArgs a) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= a.P) return;
    const int N = a.N, K = a.k;
    // row offsets of separation d: rows (a, a + d), a = 0..N-1-d
    int off[kNet];
    {
        int o = 0;
#pragma unroll
        for (int d = 1; d <= kNet; ++d) {
            off[d - 1] = o;
            o += d <= K && N - d > 0 ? N - d : 0;
        }
    }
    float bb[kNet][BREG ? NX : 1], z[kNet][NX], u[kNet][NX], x[NX];
    // interferogram (i, i + d), zero on rows outside the network of N dates
    auto bval = [&](int d, int i) __attribute__((always_inline)) -> float {
        const bool v = d <= K && i + d <= N - 1;
        if constexpr (BREG) {
            return bb[d - 1][i];
        } else {
            const float* src = a.b + (int64_t)(v ? off[d - 1] + i : 0) * a.P + p;
            const float w = *src;
            return v ? w : 0.f;
        }
    };
#pragma unroll
    for (int d = 1; d <= kNet; ++d)
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            if constexpr (BREG) {
                const bool v = d <= K && i + d <= N - 1;
                bb[d - 1][i] = v ? a.b[(int64_t)(off[d - 1] + i) * a.P + p] : 0.f;
            }
            z[d - 1][i] = 0.f;
            u[d - 1][i] = 0.f;
        }
#pragma unroll
    for (int c = 0; c < NX; ++c) x[c] = 0.f;
    for (int it = 0; it < a.iters; ++it) {
        // w = A^T (b + z - u); pair (i, i + d): +v at date i + d, -v at date i
        float w[NX];
#pragma unroll
        for (int c = 0; c < NX; ++c) w[c] = 0.f;
#pragma unroll
        for (int d = 1; d <= kNet; ++d)
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                if (i + d > NX) continue;
                const float v = bval(d, i) + z[d - 1][i] - u[d - 1][i];  // zero on unused rows
                w[i + d - 1] += v;
                if (i >= 1) w[i - 1] -= v;
            }
        // L y = w, then L^T x = y (dates beyond N - 1: identity rows, w = 0)
#pragma unroll
        for (int c = 0; c < NX; ++c) {
            float s = w[c];
#pragma unroll
            for (int d = 1; d <= kNet; ++d)
                if (c - d >= 0) s -= a.sub[d - 1][c] * x[c - d];
            x[c] = s * a.inv_diag[c];
        }
#pragma unroll
        for (int c = NX - 1; c >= 0; --c) {
            float s = x[c];
#pragma unroll
            for (int d = 1; d <= kNet; ++d)
                if (c + d < NX) s -= a.sub[d - 1][c + d] * x[c + d];
            x[c] = s * a.inv_diag[c];
        }
#pragma unroll
        for (int d = 1; d <= kNet; ++d)
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                if (i + d > NX) continue;
                const bool v = d <= K && i + d <= N - 1;
                const float ax = x[i + d - 1] - (i >= 1 ? x[i - 1] : 0.f);
                const float t = ax - bval(d, i) + u[d - 1][i];
                const float zz = t > a.kappa ? t - a.kappa : (t < -a.kappa ? t + a.kappa : 0.f);
                z[d - 1][i] = v ? zz : 0.f;
                u[d - 1][i] = v ? t - zz : 0.f;
            }
    }
#pragma unroll
    for (int c = 0; c < NX; ++c)
        if (c < N - 1) a.x[(int64_t)c * a.P + p] = x[c];
    if (a.resid) {
        float r = 0.f;
#pragma unroll
        for (int d = 1; d <= kNet; ++d)
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                if (i + d > NX) continue;
                const bool v = d <= K && i + d <= N - 1;
                const float ax = x[i + d - 1] - (i >= 1 ? x[i - 1] : 0.f);
                r += v ? fabsf(ax - bval(d, i)) : 0.f;
            }
        a.resid[p] = r;
    }
}

}  // namespace
}  // namespace plk

using namespace plk;

#define PL_CHECK(cond, status, ...) \
    do {                            \
        if (!(cond)) return fail(status, __VA_ARGS__); \
    } while (0)

extern "C" {

pl_status pl_ps_regrid(const pl_c64* stack, int32_t N, int64_t R, int64_t C, pl_window w, int32_t ref_idx,
                       const double* mean, const double* var, double da_threshold, const pl_c64* ds_phasors,
                       pl_c64* out_phasors, int64_t* ps_source, uint8_t* ps_mask, pl_stream stream) {
    Geometry g;
    PL_CHECK(stack && mean && var && ds_phasors && out_phasors, PL_ERR_INVALID_ARG, "pl_ps_regrid: NULL pointer");
    PL_CHECK(N >= 1 && N <= kMaxN, PL_ERR_UNSUPPORTED, "pl_ps_regrid: N=%d outside 1..%d", N, kMaxN);
    PL_CHECK(make_geometry(R, C, w, &g), PL_ERR_SHAPE, "pl_ps_regrid: bad image size or window");
    PL_CHECK(g.oR >= 1 && g.oC >= 1, PL_ERR_SHAPE, "pl_ps_regrid: image smaller than one stride");
    PL_CHECK(ref_idx >= 0 && ref_idx < N, PL_ERR_INVALID_ARG, "pl_ps_regrid: ref_idx %d outside 0..%d", ref_idx,
             N - 1);
    PL_CHECK(da_threshold >= 0 && std::isfinite(da_threshold), PL_ERR_INVALID_ARG,
             "pl_ps_regrid: threshold must be finite and >= 0");
    const int64_t P = g.oR * g.oC;
    PL_CHECK((P + kBlock - 1) / kBlock <= 2147483647LL, PL_ERR_UNSUPPORTED, "pl_ps_regrid: output grid too large");
    RegridArgs a{contiguous_planes(stack, N, R * C), N, ref_idx, g, mean, var, da_threshold,
                 reinterpret_cast<const float2*>(ds_phasors), reinterpret_cast<float2*>(out_phasors), ps_source,
                 ps_mask};
    hipLaunchKernelGGL(ps_regrid_kernel, dim3((unsigned)((P + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       reinterpret_cast<hipStream_t>(stream), a);
    return launch_ok("PS regridding kernel");
}

pl_status pl_phase_similarity(const pl_c64* phasors, int32_t N, int64_t oR, int64_t oC, const uint8_t* flags,
                              int32_t radius, int32_t k, float* gamma_s, pl_stream stream) {
    PL_CHECK(phasors && gamma_s, PL_ERR_INVALID_ARG, "pl_phase_similarity: NULL pointer");
    PL_CHECK(N >= 1 && N <= kMaxN, PL_ERR_UNSUPPORTED, "pl_phase_similarity: N=%d outside 1..%d", N, kMaxN);
    PL_CHECK(oR >= 1 && oC >= 1, PL_ERR_SHAPE, "pl_phase_similarity: empty grid");
    PL_CHECK(radius >= 1 && (2 * radius + 1) * (2 * radius + 1) <= 64 * kSimSlots, PL_ERR_UNSUPPORTED,
             "pl_phase_similarity: radius %d outside 1..15", radius);
    PL_CHECK(k >= 1 && k <= kNet, PL_ERR_UNSUPPORTED, "pl_phase_similarity: network of %d neighbours (1..3)", k);
    const int64_t P = oR * oC;
    const int64_t blocks = (P + kBlock / 64 - 1) / (kBlock / 64);
    PL_CHECK(blocks <= 2147483647LL, PL_ERR_UNSUPPORTED, "pl_phase_similarity: grid too large");
    SimArgs a{reinterpret_cast<const float2*>(phasors), flags, oR, oC, N, k, radius, gamma_s};
    hipLaunchKernelGGL(phase_similarity_kernel, dim3((unsigned)blocks), dim3(kBlock), 0,
                       reinterpret_cast<hipStream_t>(stream), a);
    return launch_ok("phase similarity kernel");
}

pl_status pl_network_size(int32_t N, int32_t k, int32_t* n_ifg) {
    PL_CHECK(n_ifg, PL_ERR_INVALID_ARG, "pl_network_size: NULL output");
    PL_CHECK(N >= 2 && N <= kMaxN, PL_ERR_UNSUPPORTED, "pl_network_size: N=%d outside 2..%d", N, kMaxN);
    PL_CHECK(k >= 1 && k <= kNet, PL_ERR_UNSUPPORTED, "pl_network_size: k=%d outside 1..3", k);
    int n = 0;
    for (int d = 1; d <= k; ++d) n += N - d > 0 ? N - d : 0;
    *n_ifg = n;
    return PL_OK;
}

pl_status pl_network_invert_l1(const float* ifg, int32_t N, int32_t k, int64_t P, double rho, int32_t iters,
                               float* x, float* residual_l1, pl_stream stream) {
    int32_t nifg = 0;
    pl_status st = pl_network_size(N, k, &nifg);
    if (st != PL_OK) return st;
    PL_CHECK(P >= 0, PL_ERR_SHAPE, "pl_network_invert_l1: negative pixel count");
    PL_CHECK(P == 0 || (ifg && x), PL_ERR_INVALID_ARG, "pl_network_invert_l1: NULL pointer");
    PL_CHECK(rho > 0 && std::isfinite(rho), PL_ERR_INVALID_ARG, "pl_network_invert_l1: rho must be > 0");
    PL_CHECK(iters >= 0, PL_ERR_INVALID_ARG, "pl_network_invert_l1: negative iteration count");
    PL_CHECK((P + kBlock - 1) / kBlock <= 2147483647LL, PL_ERR_UNSUPPORTED, "pl_network_invert_l1: too many pixels");
    if (P == 0) return PL_OK;
    // A^T A of the network (dates 1..N-1; date 0 is the reference), factored
    // in FP64 on the host: a banded Cholesky factor of bandwidth k
    const int n = N - 1;
    std::vector<double> M((size_t)n * n, 0.0), L((size_t)n * n, 0.0);
    for (int d = 1; d <= k; ++d)
        for (int i = 0; i + d <= N - 1; ++i) {
            const int e = i + d - 1, s = i - 1;  // columns of dates i + d and i
            M[(size_t)e * n + e] += 1.0;
            if (s >= 0) {
                M[(size_t)s * n + s] += 1.0;
                M[(size_t)e * n + s] -= 1.0;
                M[(size_t)s * n + e] -= 1.0;
            }
        }
    for (int c = 0; c < n; ++c) {
        for (int j = 0; j <= c; ++j) {
            double v = M[(size_t)c * n + j];
            for (int m = 0; m < j; ++m) v -= L[(size_t)c * n + m] * L[(size_t)j * n + m];
            if (j == c) {
                PL_CHECK(v > 0, PL_ERR_INVALID_ARG, "pl_network_invert_l1: network matrix not positive definite");
                L[(size_t)c * n + c] = std::sqrt(v);
            } else {
                L[(size_t)c * n + j] = v / L[(size_t)j * n + j];
            }
        }
    }
    AdmmArgs a{};
    a.b = ifg;
    a.x = x;
    a.resid = residual_l1;
    a.P = P;
    a.N = N;
    a.k = k;
    a.iters = iters;
    a.kappa = (float)(1.0 / rho);
    for (int c = 0; c < kMaxN; ++c) {
        a.inv_diag[c] = c < n ? (float)(1.0 / L[(size_t)c * n + c]) : 1.f;
        for (int d = 1; d <= kNet; ++d)
            a.sub[d - 1][c] = (c < n && c - d >= 0) ? (float)L[(size_t)c * n + c - d] : 0.f;
    }
    const dim3 grid((unsigned)((P + kBlock - 1) / kBlock)), block(kBlock);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (N <= 16) hipLaunchKernelGGL((admm_kernel<15, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((admm_kernel<31, false>), grid, block, 0, s, a);
    return launch_ok("ADMM inversion kernel");
}

}  // extern "C"
