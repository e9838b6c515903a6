// Adjoint of the sample coherence and EMI / EVD phase linking (Sec. 2.1
// eq. sample-coherence, Sec. 3.2 eq. emi-eigenvalue-problem), with the SHP
// mask and the EMI/EVD choice held fixed.
//
// link_vjp_kernel, one pixel per group of NP lanes (lane i = row i), with
// A = sum z z^H over the SHPs, d = diag(A), C = D^-1/2 A D^-1/2, G = |C|,
// H = G^-1 o C (EMI) or -C (EVD), (v, lambda) its smallest eigenpair and
// g = dL/dphi:
//  1. the eigenpair is recomputed by the forward solver;
//  2. phi_i = Im log(v_i conj(v_r)) gives dL = Re(u^H dv) with
//     u_i = j conj(w_i), w_i = g_i / v_i (i != r), w_r = -(sum_{i!=r} g_i) / v_r;
//  3. dv = -(H - lambda I)^+ dH v, so Hbar = -y v^H with
//     y = (H - lambda I)^+ u, formed as (H - lambda I + v v^H)^{-1} (u - v v^H u)
//     (the added term moves the zero eigenvalue to 1 and leaves the other
//     eigenvectors alone); Hbar is replaced by its Hermitian part since dH is
//     Hermitian;
//  4. EMI: Kbar = Re(conj(Hbar) o C), Gbar = -G^-1 Kbar G^-1 (FP64),
//     Cbar = Hbar o G^-1 + Gbar o C / |C|;  EVD: Cbar = -Hbar;
//  5. Abar = Cbar / sqrt(d d^T) with Abar_ii -= sum_j Re(conj(Cbar_ij) C_ij) / d_i
//     (the normalisation's dependence on d_i through row and column i);
//  6. S = Abar + Abar^H = 2 Abar is written as its upper triangle,
//     entry-major [N(N+1)/2][P] so that the gather reads it coalesced.
//
// vjp_gather_kernel, one thread per input pixel q: grad z_q = T_q z_q with
// T_q = sum of S_p over the output pixels p whose window holds q as an SHP.
// The candidate p form a box of at most (2 h_y / s_y + 1) x (2 h_x / s_x + 1)
// output pixels; each thread keeps a bitset of its SHP memberships in LDS and
// sums one entry plane at a time over it, so a wavefront re-reads a small
// 2-D patch of the plane from L1.
#include <cmath>

#include "eig_device.hpp"

namespace plk {
namespace {

struct VjpArgs {
    const float2* coh;
    const float* diag;
    const uint8_t* flags;
    const float* grad;  // [N][P]
    int N;
    int64_t npix;
    int ref;
    float2* S;          // [N(N+1)/2][P]
};

// upper-triangle entry index of (m, n), m <= n < N
__device__ __forceinline__ int tri_index(int m, int n, int N) { return m * N - (m * (m - 1)) / 2 + (n - m); }

template <int NP, int NJ>
__global__ __launch_bounds__(kBlock) void link_vjp_kernel(VjpArgs a) {
    constexpr int GPW = 64 / NP;
    constexpr int ROW_BYTES = (NJ + 2) * 8;
    constexpr int GROUP_BYTES = 2 * ROW_BYTES + NP * 8;
    __shared__ __attribute__((aligned(16))) unsigned char lds[(kBlock / 64) * GPW * GROUP_BYTES];
    // per lane one row of NJ 8-byte slots: B (float2) during the eigen-solve,
    // then G^-1 and G^-1 Kbar rows (double)
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
    float2* bme = &brow[0][threadIdx.x];                       // this lane's slot j at bme[j * kBlock]
    double* dme = reinterpret_cast<double*>(bme);              // same slots as double
    const double* dgrp = reinterpret_cast<const double*>(&brow[0][threadIdx.x - i]);  // lane l of the group: dgrp[j * kBlock + l]

    const int N = a.N;
    const int64_t P = a.npix;
    const int64_t pix = ((int64_t)blockIdx.x * (kBlock / 64) + wave) * GPW + grp;
    const bool active = pix < P;
    const bool row_live = active && i < N;
    const uint8_t flag = active ? a.flags[pix] : (uint8_t)PL_FLAG_INVALID;
    const bool emi = flag == PL_FLAG_EMI;

    // ---- row i of C and d_i
    const float2* src = a.coh + (active ? pix : 0) * (int64_t)N * N + (int64_t)i * N;
    float2 c[NJ];
#pragma unroll NJ
    for (int j = 0; j < NJ; ++j) c[j] = (row_live && j < N) ? src[j] : make_float2(0.f, 0.f);
    const float di = row_live ? a.diag[pix * N + i] : 1.f;
    bool bad = row_live && !(di > 0.f && di <= 3.4e38f);
#pragma unroll NJ
    for (int j = 0; j < NJ; ++j) bad = bad || !(fabsf(c[j].x) <= 3.4e38f && fabsf(c[j].y) <= 3.4e38f);
    bool skip = !active || flag == PL_FLAG_INVALID || gany<NP>(bad, grp);

    float2 x = make_float2(0.f, 0.f);
#pragma unroll NJ
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
        const float s = 1.0f / sqrtf(nrm);
        x.x *= s;
        x.y *= s;
    }
    float evd_shift;
    {
        float rs = 0.f;
#pragma unroll NJ
        for (int j = 0; j < NJ; ++j) rs += sqrtf(c[j].x * c[j].x + c[j].y * c[j].y);
        evd_shift = -(1.0f + 1e-3f) * gmax<NP>(rs) - 1e-3f;
    }

    // ---- 1. the forward eigen-solve on the same C
    double gi[NJ];
#pragma unroll NJ
    for (int j = 0; j < NJ; ++j) {
        gi[j] = (row_live && j < N) ? cabs64(c[j].x, c[j].y) : 0.0;
    }
    // an EMI pixel whose |C| no longer inverts cannot be differentiated on the
    // EMI branch: it contributes nothing
    const bool gfail = invert_g<NJ>(gi, N, i, emi && !skip, rbd0, rbd1);
    skip = skip || (emi && gfail);
    float bnorm2 = 0.f;
#pragma unroll NJ
    for (int j = 0; j < NJ; ++j) {
        float2 v;
        if (!emi) v = make_float2(-c[j].x, -c[j].y);
        else v = make_float2((float)gi[j] * c[j].x, (float)gi[j] * c[j].y);
        bme[j * kBlock] = v;
        bnorm2 += v.x * v.x + v.y * v.y;
    }
    float2 m[1][NJ];
    bool conv;
    int it, retries;
    {
        float2 xv[1] = {x};
        eig_min<NP, NJ>(m, bme, bnorm2, emi ? 0.99f : evd_shift, !skip, N, i, rbc0, rbc1, xb, xv, conv, it,
                        retries);
        x = xv[0];
    }
    const float2 bx = matvec_lds<NJ>(bme, x, i, xb);
    const float lam = gsum<NP>(x.x * bx.x + x.y * bx.y);

    // ---- 2. u
    const float gph = row_live ? a.grad[(int64_t)i * P + pix] : 0.f;
    const float gtot = gsum<NP>(gph);
    const float x2 = x.x * x.x + x.y * x.y;
    const float num = (i == a.ref) ? -(gtot - gph) : gph;
    float2 u = make_float2(0.f, 0.f);
    if (row_live && x2 > 1e-30f) {
        const float2 w = make_float2(num * x.x / x2, -num * x.y / x2);  // num / x_i
        u = make_float2(w.y, w.x);                                        // j conj(w)
    }
    // ---- 3. y = (H - lambda I + v v^H)^{-1} (u - v v^H u)
    {
        const float sr = gsum<NP>(x.x * u.x + x.y * u.y), si = gsum<NP>(x.x * u.y - x.y * u.x);  // v^H u
        u.x -= x.x * sr - x.y * si;
        u.y -= x.x * si + x.y * sr;
    }
    xb[i] = x;
    float2 mv[NJ];
#pragma unroll NJ
    for (int j = 0; j < NJ; ++j) {
        const float2 b = bme[j * kBlock], xj = xb[j];
        // B_ij + x_i conj(x_j)
        mv[j] = make_float2(b.x + x.x * xj.x + x.y * xj.y, b.y + x.y * xj.x - x.x * xj.y);
    }
    invert_c<NJ>(mv, lam, N, i, !skip, rbc0, rbc1);
    float2 y = matvec<NJ>(mv, u, i, xb);
    {
        const float sr = gsum<NP>(x.x * y.x + x.y * y.y), si = gsum<NP>(x.x * y.y - x.y * y.x);
        y.x -= x.x * sr - x.y * si;
        y.y -= x.x * si + x.y * sr;
    }
    if (skip || !row_live) y = make_float2(0.f, 0.f);
    // Hbar_ij = -(y_i conj(x_j) + x_i conj(y_j)) / 2 (Hermitian part of -y x^H)
    auto hbar = [&](int j) {
        const float2 xj = xb[j], yj = rbc1[j];
        return make_float2(-0.5f * (y.x * xj.x + y.y * xj.y + x.x * yj.x + x.y * yj.y),
                           -0.5f * (y.y * xj.x - y.x * xj.y + x.y * yj.x - x.x * yj.y));
    };

    // ---- 4. Cbar and t_i = sum_j Re(conj(Cbar_ij) C_ij).  C is read again
    // (an L2 hit) and |C|^{-1} recomputed rather than kept live through the
    // eigen-solve.
#pragma unroll NJ
    for (int j = 0; j < NJ; ++j) c[j] = (row_live && j < N) ? src[j] : make_float2(0.f, 0.f);
    if (emi) {
#pragma unroll NJ
        for (int j = 0; j < NJ; ++j) {
            gi[j] = (row_live && j < N) ? cabs64(c[j].x, c[j].y) : 0.0;
        }
    }
    invert_g<NJ>(gi, N, i, emi && !skip, rbd0, rbd1);
    // broadcast x (xb) and y (rbc1; the pivot-row buffers are free from here on)
    xb[i] = x;
    if (i < NJ) rbc1[i] = y;
    float trow = 0.f;
    if (emi) {
        // Kbar_ij = Re(conj(Hbar_ij) C_ij) into this lane's LDS slots
#pragma unroll NJ
        for (int j = 0; j < NJ; ++j) {
            const float2 h = hbar(j);
            dme[j * kBlock] = (double)h.x * c[j].x + (double)h.y * c[j].y;
        }
        // w = (G^-1)_i Kbar, i.e. w_l = sum_k G^-1_ik Kbar_kl
        double w[NJ];
#pragma unroll NJ
        for (int l = 0; l < NJ; ++l) w[l] = 0.0;
#pragma unroll NJ
        for (int k = 0; k < NJ; ++k) {
            if (k < N) {
#pragma unroll NJ
                for (int l = 0; l < NJ; ++l) w[l] = fma(gi[k], dgrp[l * kBlock + k], w[l]);
            }
        }
        // rows of G^-1 replace Kbar in LDS (every read of Kbar above precedes
        // these writes in the wavefront's program order)
#pragma unroll NJ
        for (int j = 0; j < NJ; ++j) dme[j * kBlock] = gi[j];
        // Gbar_ij = -sum_l w_l G^-1_lj
        double t[NJ];
#pragma unroll NJ
        for (int j = 0; j < NJ; ++j) t[j] = 0.0;
#pragma unroll NJ
        for (int l = 0; l < NJ; ++l) {
            if (l < N) {
#pragma unroll NJ
                for (int j = 0; j < NJ; ++j) t[j] = fma(-w[l], dgrp[j * kBlock + l], t[j]);
            }
        }
#pragma unroll NJ
        for (int j = 0; j < NJ; ++j) c[j] = (row_live && j < N) ? src[j] : make_float2(0.f, 0.f);
#pragma unroll NJ
        for (int j = 0; j < NJ; ++j) {
            const float2 h = hbar(j);
            const float ac = sqrtf(c[j].x * c[j].x + c[j].y * c[j].y);
            const float gij = (float)dme[j * kBlock];
            const float gb = (float)t[j];
            float2 cb = make_float2(h.x * gij, h.y * gij);
            if (ac > 0.f) {
                cb.x += gb * c[j].x / ac;
                cb.y += gb * c[j].y / ac;
            }
            trow += cb.x * c[j].x + cb.y * c[j].y;
            c[j] = cb;
        }
    } else {
#pragma unroll NJ
        for (int j = 0; j < NJ; ++j) {
            const float2 h = hbar(j);
            const float2 cb = make_float2(-h.x, -h.y);
            trow += cb.x * c[j].x + cb.y * c[j].y;
            c[j] = cb;
        }
    }

    // ---- 5./6. S = 2 Abar, upper triangle of row i
    const float isd = 1.0f / sqrtf(di);
    const float* drow = a.diag + (active ? pix : 0) * N;
    if (row_live) {
        int e = tri_index(i, i, N);
#pragma unroll NJ
        for (int j = 0; j < NJ; ++j) {
            if (j >= i && j < N) {
                const float sc = 2.0f * isd / sqrtf(drow[j]);
                float2 s = make_float2(c[j].x * sc, c[j].y * sc);
                if (j == i) s.x -= 2.0f * trow / di;
                if (skip) s = make_float2(0.f, 0.f);
                a.S[(int64_t)e * P + pix] = s;
                ++e;
            }
        }
    }
}

struct GatherArgs {
    PlaneTable t;
    int N;
    Geometry g;
    const uint32_t* mask;
    const float2* S;
    float2* grad;
    int ny, nx;   // candidate box of output pixels per input pixel
    int nwc;      // 32-bit words of the candidate bitset
};

constexpr int kGatherX = 64, kGatherY = 4;
constexpr int kMaxCandWords = PL_MAX_WINDOW / 32;

template <int NJ>
__global__ __launch_bounds__(kGatherX * kGatherY) void vjp_gather_kernel(GatherArgs a) {
    __shared__ uint32_t bits[kMaxCandWords][kGatherX * kGatherY];
    const Geometry& g = a.g;
    const int tid = threadIdx.y * kGatherX + threadIdx.x;
    const int64_t qx = (int64_t)blockIdx.x * kGatherX + threadIdx.x;
    const int64_t qy = (int64_t)blockIdx.y * kGatherY + threadIdx.y;
    const bool live = qx < g.C && qy < g.R;
    const int N = a.N;
    const int64_t P = g.oR * g.oC;
    // first candidate output row / column: centre o*s + s/2 >= q - h
    auto first = [](int64_t q, int h, int s) {
        const int64_t lo = q - h - s / 2;
        return lo <= 0 ? (int64_t)0 : (lo + s - 1) / s;
    };
    const int64_t oy0 = first(qy, g.hy, g.sy), ox0 = first(qx, g.hx, g.sx);
    bool any = false;
    {
        int idx = 0;
        uint32_t word = 0;
        for (int cy = 0; cy < a.ny; ++cy) {
            for (int cx = 0; cx < a.nx; ++cx, ++idx) {
                const int64_t oy = oy0 + cy, ox = ox0 + cx;
                const int64_t dy = qy - (oy * g.sy + g.sy / 2), dx = qx - (ox * g.sx + g.sx / 2);
                bool b = false;
                if (live && oy < g.oR && ox < g.oC && dy >= -g.hy && dy <= g.hy && dx >= -g.hx && dx <= g.hx) {
                    const int bit = (int)((dy + g.hy) * g.wx + (dx + g.hx));
                    b = (a.mask[(oy * g.oC + ox) * g.nw + (bit >> 5)] >> (bit & 31)) & 1u;
                }
                word |= (uint32_t)b << (idx & 31);
                any = any || b;
                if ((idx & 31) == 31) {
                    bits[idx >> 5][tid] = word;
                    word = 0;
                }
            }
        }
        if (idx & 31) bits[idx >> 5][tid] = word;
    }
    float2 z[NJ], acc[NJ];
#pragma unroll
    for (int n = 0; n < NJ; ++n) {
        z[n] = make_float2(0.f, 0.f);
        acc[n] = make_float2(0.f, 0.f);
        if (n < N && live && any) z[n] = a.t.p[n][qy * g.C + qx];
    }
    const int64_t pbase = oy0 * g.oC + ox0;
    int e = 0;
#pragma unroll
    for (int mm = 0; mm < NJ; ++mm) {
#pragma unroll
        for (int nn = mm; nn < NJ; ++nn) {
            if (nn < N) {
                const float2* plane = a.S + (int64_t)e * P + pbase;
                float2 T = make_float2(0.f, 0.f);
                int idx = 0;
                uint32_t word = 0;
                for (int cy = 0; cy < a.ny; ++cy) {
                    const float2* row = plane + (int64_t)cy * g.oC;
                    for (int cx = 0; cx < a.nx; ++cx, ++idx) {
                        if ((idx & 31) == 0) word = bits[idx >> 5][tid];
                        if (word & 1u) {
                            const float2 v = row[cx];
                            T.x += v.x;
                            T.y += v.y;
                        }
                        word >>= 1;
                    }
                }
                // grad[mm] += T z[nn];  grad[nn] += conj(T) z[mm] (off-diagonal)
                acc[mm].x += T.x * z[nn].x - T.y * z[nn].y;
                acc[mm].y += T.x * z[nn].y + T.y * z[nn].x;
                if (nn != mm) {
                    acc[nn].x += T.x * z[mm].x + T.y * z[mm].y;
                    acc[nn].y += T.x * z[mm].y - T.y * z[mm].x;
                }
                ++e;
            }
        }
    }
    if (live) {
#pragma unroll
        for (int n = 0; n < NJ; ++n)
            if (n < N) a.grad[(int64_t)n * g.R * g.C + qy * g.C + qx] = acc[n];
    }
}

}  // namespace

pl_status launch_link_vjp(const float2* coh, const float* diag, const uint8_t* flags,
                          const float* grad_phase, int N, int64_t npix, int ref, float2* S,
                          hipStream_t s) {
    VjpArgs a{coh, diag, flags, grad_phase, N, npix, ref, S};
    if (npix == 0) return PL_OK;
    const int np = N <= 16 ? 16 : 32;
    const int64_t per_block = (kBlock / 64) * (64 / np);
    const int64_t blocks = (npix + per_block - 1) / per_block;
    if (blocks > 2147483647LL) return fail(PL_ERR_UNSUPPORTED, "pl_phase_link_vjp: too many pixels");
    const dim3 grid((unsigned)blocks), block(kBlock);
    switch ((N + 3) / 4) {
        case 1: case 2: case 3: hipLaunchKernelGGL((link_vjp_kernel<16, 12>), grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL((link_vjp_kernel<16, 16>), grid, block, 0, s, a); break;
        case 5: hipLaunchKernelGGL((link_vjp_kernel<32, 20>), grid, block, 0, s, a); break;
        case 6: hipLaunchKernelGGL((link_vjp_kernel<32, 24>), grid, block, 0, s, a); break;
        case 7: hipLaunchKernelGGL((link_vjp_kernel<32, 28>), grid, block, 0, s, a); break;
        default: hipLaunchKernelGGL((link_vjp_kernel<32, 32>), grid, block, 0, s, a); break;
    }
    return launch_ok("phase linking adjoint kernel");
}

pl_status launch_vjp_gather(const PlaneTable& t, int N, const Geometry& g, const uint32_t* mask,
                            const float2* S, float2* grad, hipStream_t s) {
    GatherArgs a{};
    a.t = t;
    a.N = N;
    a.g = g;
    a.mask = mask;
    a.S = S;
    a.grad = grad;
    a.ny = (2 * g.hy) / g.sy + 1;
    a.nx = (2 * g.hx) / g.sx + 1;
    a.nwc = (a.ny * a.nx + 31) / 32;
    if (a.nwc > kMaxCandWords) return fail(PL_ERR_UNSUPPORTED, "pl_phase_link_vjp: window too large");
    const int64_t gx = (g.C + kGatherX - 1) / kGatherX, gy = (g.R + kGatherY - 1) / kGatherY;
    if (gx > 2147483647LL || gy > 65535) return fail(PL_ERR_UNSUPPORTED, "pl_phase_link_vjp: image too large");
    const dim3 grid((unsigned)gx, (unsigned)gy), block(kGatherX, kGatherY);
    switch ((N + 3) / 4) {
        case 1: case 2: case 3: hipLaunchKernelGGL(vjp_gather_kernel<12>, grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL(vjp_gather_kernel<16>, grid, block, 0, s, a); break;
        case 5: hipLaunchKernelGGL(vjp_gather_kernel<20>, grid, block, 0, s, a); break;
        case 6: hipLaunchKernelGGL(vjp_gather_kernel<24>, grid, block, 0, s, a); break;
        case 7: hipLaunchKernelGGL(vjp_gather_kernel<28>, grid, block, 0, s, a); break;
        default: hipLaunchKernelGGL(vjp_gather_kernel<32>, grid, block, 0, s, a); break;
    }
    return launch_ok("adjoint gather kernel");
}

}  // namespace plk
