// FP64 adjoint of the sample coherence and EMI / EVD phase linking (Sec. 2.1
// eq. sample-coherence, Sec. 3.2 eq. emi-eigenvalue-problem), with the SHP
// mask and the EMI/EVD choice held fixed: the same derivation as the FP32
// adjoint (link_vjp.hip), every step in double precision, for gradients that
// match finite differences of an FP64 evaluation to ~1e-10.
//
// vjp64_pixel_kernel, one wavefront per output pixel, its matrices in LDS
// (lane i < N updates row i; lanes exchange rows through LDS):
//  1. A = sum over the SHPs of z z^H, accumulated from the FP32 stack in FP64
//     (every product of two FP32 values is exact in FP64), lane e owning the
//     entries e, e + 64, ... of the row-major N x N matrix;
//  2. d = diag(A), C = A / sqrt(d d^T), G = |C|, G^-1 by Gauss-Jordan (an EMI
//     pixel whose pivots are not all above 1e-6 contributes nothing);
//  3. H = G^-1 o C (EMI) or -C (EVD) and its smallest eigenpair (v, lambda)
//     by shifted inverse iteration, each shift validated by the inertia of
//     (H - mu I) (all Gauss-Jordan pivots positive) and moved up to the
//     Rayleigh quotient minus twice the residual while it converges slowly;
//  4. u from dL/dphi (u_i = j conj(w_i), w_i = g_i / v_i, w_r = -sum g / v_r),
//     y = (H - lambda I + v v^H)^{-1} (u - v v^H u), projected off v;
//     Hbar = Hermitian part of -y v^H;
//  5. EMI: Kbar = Re(conj(Hbar) o C), Gbar = -G^-1 Kbar G^-1,
//     Cbar = Hbar o G^-1 + Gbar o C / |C|;  EVD: Cbar = -Hbar;
//  6. S = 2 Abar, Abar = Cbar / sqrt(d d^T) - diag(sum_j Re(conj(Cbar_ij) C_ij) / d_i),
//     its upper triangle written entry-major [N(N+1)/2][P] (double2).
// vjp64_gather_kernel: grad z_q = sum over the windows holding q of S_p z_q,
// accumulated in FP64, written as complex64.
#include <cmath>

#include "internal.hpp"

namespace plk {
namespace {

constexpr int kLD = kMaxN + 1;   // row pitch of the LDS matrices (entries)
constexpr double kTau = 1e-6;    // LDL^T pivot below which |C| does not invert
constexpr int kMaxIter64 = 400;

struct V64Args {
    PlaneTable t;
    int N;
    Geometry g;
    const uint32_t* mask;
    const uint8_t* flags;
    const float* grad;  // [N][P]
    int ref;
    double2* S;         // [N(N+1)/2][P]
};

struct Lds64 {
    double2 C[kMaxN * kLD];   // C, later Cbar
    double2 W[kMaxN * kLD];   // H - mu I and its inverse; H - lambda I + v v^H and its inverse
    double2 H[kMaxN * kLD];   // H
    double Gi[kMaxN * kLD];   // G^-1, later Kbar rows
    double2 z[kMaxN];         // staged sample; vectors
    double2 x[kMaxN];
    double2 y[kMaxN];
    double piv[kMaxN];
};

__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double2 cm(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmc(double2 a, double2 b) {  // a conj(b)
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// In-place Gauss-Jordan inverse of the real N x N matrix M (lane i < N owns
// row i); returns whether every pivot was > tau and finite.
__device__ bool gj_real(double* M, double* piv, int N, int lane, double tau) {
    bool ok = true;
    for (int k = 0; k < N; ++k) {
        const double p = M[k * kLD + k];
        ok = ok && p > tau && p <= 1.7976931348623157e308;
        const double rp = 1.0 / p;
        wsync();
        if (lane == k) {
            for (int j = 0; j < N; ++j) M[k * kLD + j] *= rp;
            M[k * kLD + k] = rp;
        }
        wsync();
        if (lane < N && lane != k) {
            const double f = M[lane * kLD + k];
            M[lane * kLD + k] = 0.0;
            for (int j = 0; j < N; ++j) M[lane * kLD + j] = fma(-f, M[k * kLD + j], M[lane * kLD + j]);
        }
        wsync();
    }
    (void)piv;
    return ok;
}

// In-place Gauss-Jordan inverse of the complex Hermitian N x N matrix M
// (unpivoted); returns whether every pivot was real-part positive and
// finite, which for a Hermitian matrix proves it positive definite.
__device__ bool gj_complex(double2* M, int N, int lane) {
    bool ok = true;
    for (int k = 0; k < N; ++k) {
        const double2 p = M[k * kLD + k];
        ok = ok && p.x > 0.0 && p.x <= 1.7976931348623157e308;
        const double d = p.x * p.x + p.y * p.y;
        const double2 rp = make_double2(p.x / d, -p.y / d);
        wsync();
        if (lane == k) {
            for (int j = 0; j < N; ++j) M[k * kLD + j] = cm(M[k * kLD + j], rp);
            M[k * kLD + k] = rp;
        }
        wsync();
        if (lane < N && lane != k) {
            const double2 f = M[lane * kLD + k];
            M[lane * kLD + k] = make_double2(0.0, 0.0);
            for (int j = 0; j < N; ++j) {
                const double2 r = cm(f, M[k * kLD + j]);
                M[lane * kLD + j] = make_double2(M[lane * kLD + j].x - r.x, M[lane * kLD + j].y - r.y);
            }
        }
        wsync();
    }
    return ok;
}

// y_i = sum_j M_ij v_j for lane i < N (v in LDS)
__device__ __forceinline__ double2 matvec64(const double2* M, const double2* v, int N, int lane) {
    double2 s = make_double2(0.0, 0.0);
    if (lane < N)
        for (int j = 0; j < N; ++j) {
            const double2 r = cm(M[lane * kLD + j], v[j]);
            s.x += r.x;
            s.y += r.y;
        }
    return s;
}

// W = H - mu I, inverted in place; true when mu < lambda_min (inertia)
__device__ bool factor_shift(Lds64& L, int N, int lane, double mu) {
    wsync();
    if (lane < N)
        for (int j = 0; j < N; ++j) {
            double2 h = L.H[lane * kLD + j];
            if (j == lane) h.x -= mu;
            L.W[lane * kLD + j] = h;
        }
    wsync();
    return gj_complex(L.W, N, lane);
}

__global__ __launch_bounds__(64) void vjp64_pixel_kernel(V64Args a) {
    __shared__ Lds64 L;
    const int lane = threadIdx.x;
    const Geometry& g = a.g;
    const int N = a.N;
    const int64_t P = g.oR * g.oC;
    const int64_t pix = blockIdx.x;
    const uint8_t flag = a.flags[pix];
    const int tri = N * (N + 1) / 2;
    auto write_zero = [&]() {
        for (int e = lane; e < tri; e += 64) a.S[(int64_t)e * P + pix] = make_double2(0.0, 0.0);
    };
    if (flag == PL_FLAG_INVALID) {
        write_zero();
        return;
    }
    const bool emi = flag == PL_FLAG_EMI;
    // ---- 1. A over the SHPs
    const int64_t oy = pix / g.oC, ox = pix - oy * g.oC;
    const int64_t cy = oy * g.sy + g.sy / 2, cx = ox * g.sx + g.sx / 2;
    constexpr int kEnt = (kMaxN * kMaxN + 63) / 64;
    double2 acc[kEnt];
#pragma unroll
    for (int t = 0; t < kEnt; ++t) acc[t] = make_double2(0.0, 0.0);
    const uint32_t* mw = a.mask + pix * g.nw;
    for (int b = 0; b < g.W; ++b) {
        if (!((mw[b >> 5] >> (b & 31)) & 1u)) continue;  // uniform: one pixel per wavefront
        const int dy = b / g.wx - g.hy, dx = b % g.wx - g.hx;
        const int64_t qy = cy + dy, qx = cx + dx;
        if (qy < 0 || qy >= g.R || qx < 0 || qx >= g.C) continue;
        wsync();
        if (lane < N) {
            const float2 v = a.t.p[lane][qy * g.C + qx];
            L.z[lane] = make_double2((double)v.x, (double)v.y);
        }
        wsync();
#pragma unroll
        for (int t = 0; t < kEnt; ++t) {
            const int e = lane + 64 * t;
            if (e < N * N) {
                const int i = e / N, j = e - (e / N) * N;
                const double2 zi = L.z[i], zj = L.z[j];
                acc[t].x = fma(zi.x, zj.x, fma(zi.y, zj.y, acc[t].x));  // z_i conj(z_j)
                acc[t].y = fma(zi.y, zj.x, fma(-zi.x, zj.y, acc[t].y));
            }
        }
    }
    wsync();
#pragma unroll
    for (int t = 0; t < kEnt; ++t) {
        const int e = lane + 64 * t;
        if (e < N * N) L.C[(e / N) * kLD + e % N] = acc[t];
    }
    wsync();
    // ---- 2. d, C, G^-1
    const double di = lane < N ? L.C[lane * kLD + lane].x : 1.0;
    const bool bad = lane < N && !(di > 0.0 && di <= 1.7976931348623157e308);
    if (__ballot(bad)) {
        write_zero();
        return;
    }
    if (lane < N) L.piv[lane] = di;
    wsync();
    if (lane < N) {
        const double isd = 1.0 / sqrt(di);
        for (int j = 0; j < N; ++j) {
            const double s = isd / sqrt(L.piv[j]);
            double2 c = L.C[lane * kLD + j];
            c = make_double2(c.x * s, c.y * s);
            if (j == lane) c = make_double2(1.0, 0.0);
            L.C[lane * kLD + j] = c;
            L.Gi[lane * kLD + j] = sqrt(c.x * c.x + c.y * c.y);
        }
    }
    wsync();
    if (emi) {
        const bool ok = gj_real(L.Gi, L.piv, N, lane, kTau);
        if (!ok) {  // |C| no longer inverts: the EMI branch has no derivative here
            write_zero();
            return;
        }
    }
    // ---- 3. H and its smallest eigenpair
    double rowsum = 0.0;
    if (lane < N)
        for (int j = 0; j < N; ++j) {
            const double2 c = L.C[lane * kLD + j];
            const double gij = L.Gi[lane * kLD + j];
            const double2 h = emi ? make_double2(gij * c.x, gij * c.y) : make_double2(-c.x, -c.y);
            L.H[lane * kLD + j] = h;
            rowsum += sqrt(h.x * h.x + h.y * h.y);
        }
    double hmax = rowsum;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) hmax = fmax(hmax, __shfl_xor(hmax, o, 64));
    wsync();
    // start: unit-modulus phases of column ref of C
    double2 x = make_double2(0.0, 0.0);
    if (lane < N) {
        const double2 c = L.C[lane * kLD + a.ref];
        const double n = sqrt(c.x * c.x + c.y * c.y);
        x = n > 0.0 ? make_double2(c.x / n, c.y / n) : make_double2(lane == a.ref ? 1.0 : 0.0, 0.0);
    }
    {
        const double nn = wsum(x.x * x.x + x.y * x.y);
        x = make_double2(x.x / sqrt(nn), x.y / sqrt(nn));
    }
    // first shift: 0.99 (EMI, Sec. 3.2) or below the Gershgorin bound of -C
    // (EVD); backed off until the inertia check accepts it
    double mu = emi ? 0.99 : -hmax - 1e-3;
    const double backoff[3] = {0.5, 0.0, -hmax - 1.0};
    bool okf = factor_shift(L, N, lane, mu);
    for (int s = 0; s < 3 && !okf; ++s) {
        mu = backoff[s];
        okf = factor_shift(L, N, lane, mu);
    }
    double d2prev = 0.0;
    for (int it = 0; it < kMaxIter64; ++it) {
        wsync();
        if (lane < N) L.x[lane] = x;
        wsync();
        double2 y = matvec64(L.W, L.x, N, lane);
        const double n2 = wsum(y.x * y.x + y.y * y.y);
        const double sr = wsum(x.x * y.x + x.y * y.y), si = wsum(x.x * y.y - x.y * y.x);  // x^H y
        const double s2 = sr * sr + si * si;
        // rotate by conj(s)/|s| so the iterate keeps the previous phase; scale to unit norm
        const double sc = 1.0 / (sqrt(n2) * (s2 > 0.0 ? sqrt(s2) : 1.0));
        const double2 u = s2 > 0.0 ? make_double2(sr * sc, -si * sc) : make_double2(sc, 0.0);
        y = cm(y, u);
        const double d2 = wsum((y.x - x.x) * (y.x - x.x) + (y.y - x.y) * (y.y - x.y));
        x = y;
        if (d2 < 1e-28) break;
        // slow contraction: move the shift up to rho - 2 |H x - rho x|
        if ((it % 8) == 7 && d2prev > 0.0 && d2 > 0.01 * d2prev) {
            wsync();
            if (lane < N) L.x[lane] = x;
            wsync();
            const double2 hx = matvec64(L.H, L.x, N, lane);
            const double rho = wsum(x.x * hx.x + x.y * hx.y);
            const double res = sqrt(wsum((hx.x - rho * x.x) * (hx.x - rho * x.x) + (hx.y - rho * x.y) * (hx.y - rho * x.y)));
            const double cand = rho - 2.0 * res;
            if (cand > mu) {
                if (factor_shift(L, N, lane, cand)) mu = cand;
                else factor_shift(L, N, lane, mu);
            }
        }
        d2prev = d2;
    }
    wsync();
    if (lane < N) L.x[lane] = x;
    wsync();
    const double2 hx = matvec64(L.H, L.x, N, lane);
    const double lam = wsum(x.x * hx.x + x.y * hx.y);
    // ---- 4. u, y
    const int64_t gi = (int64_t)lane * P + pix;
    const double gph = lane < N ? (double)a.grad[gi] : 0.0;
    const double gtot = wsum(gph);
    const double num = lane == a.ref ? -(gtot - gph) : gph;
    double2 uu = make_double2(0.0, 0.0);
    const double x2 = x.x * x.x + x.y * x.y;
    if (lane < N && x2 > 0.0) {
        const double2 w = make_double2(num * x.x / x2, -num * x.y / x2);  // num / x_i
        uu = make_double2(w.y, w.x);                                        // j conj(w)
    }
    {
        const double sr = wsum(x.x * uu.x + x.y * uu.y), si = wsum(x.x * uu.y - x.y * uu.x);  // x^H u
        uu.x -= x.x * sr - x.y * si;
        uu.y -= x.x * si + x.y * sr;
    }
    // W = H - lambda I + x x^H, inverted (positive definite: eigenvalues 1 and
    // lambda_k - lambda)
    if (lane < N)
        for (int j = 0; j < N; ++j) {
            double2 h = L.H[lane * kLD + j];
            const double2 xx = cmc(x, L.x[j]);
            h.x += xx.x - (j == lane ? lam : 0.0);
            h.y += xx.y;
            L.W[lane * kLD + j] = h;
        }
    wsync();
    gj_complex(L.W, N, lane);
    wsync();
    if (lane < N) L.y[lane] = uu;
    wsync();
    double2 y = matvec64(L.W, L.y, N, lane);
    {
        const double sr = wsum(x.x * y.x + x.y * y.y), si = wsum(x.x * y.y - x.y * y.x);
        y.x -= x.x * sr - x.y * si;
        y.y -= x.x * si + x.y * sr;
    }
    wsync();
    if (lane < N) L.y[lane] = y;
    wsync();
    // Hbar_ij = -(y_i conj(x_j) + x_i conj(y_j)) / 2
    auto hbar = [&](int i, int j) {
        const double2 p = cmc(L.y[i], L.x[j]), q = cmc(L.x[i], L.y[j]);
        return make_double2(-0.5 * (p.x + q.x), -0.5 * (p.y + q.y));
    };
    // ---- 5. Cbar (into W) and t_i
    double trow = 0.0;
    if (emi) {
        // Kbar rows into H (as doubles in the real parts), then
        // w = G^-1_i Kbar, Gbar_i = -w G^-1
        if (lane < N)
            for (int j = 0; j < N; ++j) {
                const double2 h = hbar(lane, j), c = L.C[lane * kLD + j];
                L.H[lane * kLD + j] = make_double2(h.x * c.x + h.y * c.y, 0.0);
            }
        wsync();
        double wv[kMaxN];
#pragma unroll
        for (int l = 0; l < kMaxN; ++l) wv[l] = 0.0;
        if (lane < N)
            for (int k = 0; k < N; ++k) {
                const double gk = L.Gi[lane * kLD + k];
#pragma unroll
                for (int l = 0; l < kMaxN; ++l)
                    if (l < N) wv[l] = fma(gk, L.H[k * kLD + l].x, wv[l]);
            }
        if (lane < N)
            for (int j = 0; j < N; ++j) {
                double gb = 0.0;
#pragma unroll
                for (int l = 0; l < kMaxN; ++l)
                    if (l < N) gb = fma(-wv[l], L.Gi[l * kLD + j], gb);
                const double2 h = hbar(lane, j), c = L.C[lane * kLD + j];
                const double ac = sqrt(c.x * c.x + c.y * c.y);
                const double gij = L.Gi[lane * kLD + j];
                double2 cb = make_double2(h.x * gij, h.y * gij);
                if (ac > 0.0) {
                    cb.x += gb * c.x / ac;
                    cb.y += gb * c.y / ac;
                }
                trow += cb.x * c.x + cb.y * c.y;
                L.W[lane * kLD + j] = cb;
            }
    } else if (lane < N) {
        for (int j = 0; j < N; ++j) {
            const double2 h = hbar(lane, j), c = L.C[lane * kLD + j];
            const double2 cb = make_double2(-h.x, -h.y);
            trow += cb.x * c.x + cb.y * c.y;
            L.W[lane * kLD + j] = cb;
        }
    }
    wsync();
    // ---- 6. S = 2 Abar, upper triangle of row `lane`
    if (lane < N) {
        int e = lane * N - (lane * (lane - 1)) / 2;
        const double isd = 1.0 / sqrt(di);
        for (int j = lane; j < N; ++j, ++e) {
            const double2 cb = L.W[lane * kLD + j];
            const double sc = 2.0 * isd / sqrt(L.piv[j]);
            double2 s = make_double2(cb.x * sc, cb.y * sc);
            if (j == lane) s.x -= 2.0 * trow / di;
            a.S[(int64_t)e * P + pix] = s;
        }
    }
}

// ---- gather: one thread per input pixel q, FP64 accumulation over the
// output pixels whose window holds q as an SHP
struct G64Args {
    PlaneTable t;
    int N;
    Geometry g;
    const uint32_t* mask;
    const double2* S;
    float2* grad;
};

template <int NJ>
__global__ __launch_bounds__(256) void vjp64_gather_kernel(G64Args a) {
    const Geometry& g = a.g;
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= g.R * g.C) return;
    const int64_t qy = q / g.C, qx = q - qy * g.C;
    const int N = a.N;
    const int64_t P = g.oR * g.oC;
    double2 z[NJ], acc[NJ];
#pragma unroll
    for (int n = 0; n < NJ; ++n) {
        acc[n] = make_double2(0.0, 0.0);
        z[n] = make_double2(0.0, 0.0);
        if (n < N) {
            const float2 v = a.t.p[n][q];
            z[n] = make_double2(v.x, v.y);
        }
    }
    auto first = [](int64_t c, int h, int s) {
        const int64_t lo = c - h - s / 2;
        return lo <= 0 ? (int64_t)0 : (lo + s - 1) / s;
    };
    const int64_t oy0 = first(qy, g.hy, g.sy), ox0 = first(qx, g.hx, g.sx);
    for (int64_t oy = oy0; oy < g.oR && oy * g.sy + g.sy / 2 - g.hy <= qy; ++oy) {
        for (int64_t ox = ox0; ox < g.oC && ox * g.sx + g.sx / 2 - g.hx <= qx; ++ox) {
            const int64_t dy = qy - (oy * g.sy + g.sy / 2), dx = qx - (ox * g.sx + g.sx / 2);
            if (dy < -g.hy || dy > g.hy || dx < -g.hx || dx > g.hx) continue;
            const int bit = (int)((dy + g.hy) * g.wx + (dx + g.hx));
            const int64_t p = oy * g.oC + ox;
            if (!((a.mask[p * g.nw + (bit >> 5)] >> (bit & 31)) & 1u)) continue;
            int e = 0;
#pragma unroll
            for (int m = 0; m < NJ; ++m) {
#pragma unroll
                for (int n = m; n < NJ; ++n) {
                    if (m >= N || n >= N) continue;
                    const double2 T = a.S[(int64_t)e * P + p];
                    // grad[m] += T z[n]; grad[n] += conj(T) z[m] off the diagonal
                    acc[m].x += T.x * z[n].x - T.y * z[n].y;
                    acc[m].y += T.x * z[n].y + T.y * z[n].x;
                    if (n != m) {
                        acc[n].x += T.x * z[m].x + T.y * z[m].y;
                        acc[n].y += T.x * z[m].y - T.y * z[m].x;
                    }
                    ++e;
                }
            }
        }
    }
#pragma unroll
    for (int n = 0; n < NJ; ++n)
        if (n < N) a.grad[(int64_t)n * g.R * g.C + q] = make_float2((float)acc[n].x, (float)acc[n].y);
}

}  // namespace
}  // namespace plk

using namespace plk;

extern "C" {

pl_status pl_phase_link_vjp64_workspace(int32_t N, int64_t R, int64_t C, pl_window w, size_t* bytes) {
    Geometry g;
    if (!bytes) return fail(PL_ERR_INVALID_ARG, "pl_phase_link_vjp64_workspace: NULL output");
    if (N < 1 || N > kMaxN) return fail(PL_ERR_UNSUPPORTED, "pl_phase_link_vjp64_workspace: N=%d outside 1..%d", N, kMaxN);
    if (!make_geometry(R, C, w, &g) || g.oR < 1 || g.oC < 1)
        return fail(PL_ERR_SHAPE, "pl_phase_link_vjp64_workspace: bad image size or window");
    *bytes = (size_t)(N * (N + 1) / 2) * (size_t)(g.oR * g.oC) * sizeof(double2);
    return PL_OK;
}

pl_status pl_phase_link_vjp64(const pl_c64* stack, int32_t N, int64_t R, int64_t C, pl_window w,
                              const uint32_t* mask, const uint8_t* flags, int32_t ref_idx, const float* grad_phase,
                              pl_c64* grad_stack, void* workspace, size_t ws_bytes, pl_stream stream) {
    Geometry g;
    if (!stack || !mask || !flags || !grad_phase || !grad_stack || !workspace)
        return fail(PL_ERR_INVALID_ARG, "pl_phase_link_vjp64: NULL pointer");
    if (N < 1 || N > kMaxN) return fail(PL_ERR_UNSUPPORTED, "pl_phase_link_vjp64: N=%d outside 1..%d", N, kMaxN);
    if (!make_geometry(R, C, w, &g) || g.oR < 1 || g.oC < 1)
        return fail(PL_ERR_SHAPE, "pl_phase_link_vjp64: bad image size or window");
    if (ref_idx < 0 || ref_idx >= N)
        return fail(PL_ERR_INVALID_ARG, "pl_phase_link_vjp64: ref_idx %d outside 0..%d", ref_idx, N - 1);
    const int64_t P = g.oR * g.oC;
    const size_t need = (size_t)(N * (N + 1) / 2) * (size_t)P * sizeof(double2);
    if (ws_bytes < need)
        return fail(PL_ERR_WORKSPACE, "pl_phase_link_vjp64: workspace of %zu bytes, %zu needed", ws_bytes, need);
    if (P > 2147483647LL || (R * C + 255) / 256 > 2147483647LL)
        return fail(PL_ERR_UNSUPPORTED, "pl_phase_link_vjp64: image too large");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const PlaneTable t = contiguous_planes(stack, N, R * C);
    V64Args va{t, N, g, mask, flags, grad_phase, ref_idx, static_cast<double2*>(workspace)};
    hipLaunchKernelGGL(vjp64_pixel_kernel, dim3((unsigned)P), dim3(64), 0, s, va);
    pl_status r = launch_ok("FP64 adjoint kernel");
    if (r != PL_OK) return r;
    G64Args ga{t, N, g, mask, static_cast<const double2*>(workspace), reinterpret_cast<float2*>(grad_stack)};
    const dim3 grid((unsigned)((R * C + 255) / 256)), block(256);
    switch ((N + 3) / 4) {
        case 1: case 2: case 3: hipLaunchKernelGGL(vjp64_gather_kernel<12>, grid, block, 0, s, ga); break;
        case 4: hipLaunchKernelGGL(vjp64_gather_kernel<16>, grid, block, 0, s, ga); break;
        case 5: hipLaunchKernelGGL(vjp64_gather_kernel<20>, grid, block, 0, s, ga); break;
        case 6: hipLaunchKernelGGL(vjp64_gather_kernel<24>, grid, block, 0, s, ga); break;
        case 7: hipLaunchKernelGGL(vjp64_gather_kernel<28>, grid, block, 0, s, ga); break;
        default: hipLaunchKernelGGL(vjp64_gather_kernel<32>, grid, block, 0, s, ga); break;
    }
    return launch_ok("FP64 adjoint gather kernel");
}

}  // extern "C"
