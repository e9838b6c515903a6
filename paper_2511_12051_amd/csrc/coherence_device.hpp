// Device body of the windowed sample coherence (used by the coherence
// kernels and by the single-launch batched path); see coherence.hip for the
// method and the data movement.
#pragma once
#include <cmath>

#include "internal.hpp"
#include "lanes.hpp"

namespace plk {
namespace {

typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// wavefronts per workgroup (one workgroup per CU): 12 for 16-row tiles (three
// per SIMD within the register budget), 8 for 32-row tiles
template <int NT>
constexpr int kWaves = NT == 16 ? 12 : 8;
constexpr int waves_of(int nt) { return nt == 16 ? kWaves<16> : kWaves<32>; }



__device__ __forceinline__ uint32_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return u >> 16;
}

__device__ __forceinline__ float bf16_value(uint32_t h) { return __uint_as_float(h << 16); }


template <int NT>
struct Acc;
template <>
struct Acc<16> {
    typedef f32x4 T;
    static constexpr int R = 4;
    // row index of register v for this lane (column is lane % 16)
    __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <>
struct Acc<32> {
    typedef f32x16 T;
    static constexpr int R = 16;
    __device__ static int row(int lane, int v) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }
};

__device__ __forceinline__ int fast_div(int n, float inv) {  // exact for 0 <= n < 2^22
    return (int)(((float)n + 0.5f) * inv);
}

// Row staging.  An "item" is one image and one pixel pair (x0 + 2 px, +1) of
// the strip; a thread owns the items threadIdx.x + k * nthreads for the whole
// kernel, so staging a row costs no index arithmetic beyond a row offset.  A
// "unit" is one item in one row.
// Ring slot of input row y (y may be negative above the image).
__device__ __forceinline__ int ring_slot(int64_t y, int wy) {
    int s = (int)(y % wy);
    return s + (s < 0 ? wy : 0);
}

constexpr int kMaxItems = 8;

struct Items {
    int n;                     // items of this thread
    uint32_t dp[kMaxItems];    // image << 16 | pair
};

__device__ __forceinline__ Items make_items(const CohArgs& a, int nthreads) {
    Items it;
    it.n = 0;
    const int hw = a.tile_w >> 1, total = a.N * hw;
#pragma unroll
    for (int k = 0; k < kMaxItems; ++k) {
        const int idx = threadIdx.x + k * nthreads;
        it.dp[k] = 0;
        if (idx < total) {
            const int d = idx / hw;
            it.dp[k] = ((uint32_t)d << 16) | (uint32_t)(idx - d * hw);
            it.n = k + 1;
        }
    }
    return it;
}

// Units a thread keeps in registers while the current row is computed: its
// first kPfItems items in the first kPfRows new rows (static indices, so they
// stay in registers); any other unit is staged directly at commit time.
constexpr int kPfItems = 2;
template <int NT>
constexpr int kPfRows = 3;

template <int NT>
struct RowLoad {
    f32x4 v[kPfRows<NT>][kPfItems];
};

typedef __attribute__((address_space(1))) const float2 gfloat2;  // global memory
typedef __attribute__((address_space(1))) const f32x4 gf32x4;

// `plane` is the unit's image plane (planes[dp >> 16]), in global memory
// (the explicit address space keeps the loads global loads even when the
// pointer went through an opaque register copy).
__device__ __forceinline__ f32x4 fetch_unit_at(const CohArgs& a, const float2* plane, uint32_t dp, int64_t y,
                                              int64_t x0) {
    const Geometry& g = a.g;
    const int px = (int)(dp & 0xffffu);
    const int64_t x = x0 + 2 * px;
    f32x4 z = {0.f, 0.f, 0.f, 0.f};
    if (y >= 0 && y < g.R) {
        gfloat2* row = (gfloat2*)plane + y * g.C;
        if (a.vec_rows && x >= 0 && x + 1 < g.C) {
            z = *reinterpret_cast<gf32x4*>(row + x);  // 16-byte aligned pair
        } else {
            if (x >= 0 && x < g.C) {
                z[0] = row[x].x;
                z[1] = row[x].y;
            }
            if (x + 1 >= 0 && x + 1 < g.C) {
                z[2] = row[x + 1].x;
                z[3] = row[x + 1].y;
            }
        }
    }
    return z;
}

__device__ __forceinline__ f32x4 fetch_unit(const CohArgs& a, const float2* const* planes, uint32_t dp, int64_t y,
                                           int64_t x0) {
    return fetch_unit_at(a, planes[dp >> 16], dp, y, x0);
}

// Image planes of a thread's prefetched items, read from the plane table once
// per kernel: the table sits in argument memory and a per-lane index makes
// each read a vector memory load, which would otherwise put a dependent
// round trip (and a wait for every load in flight) before each prefetch.
struct ItemPlanes {
    const float2* p[kPfItems];
};

__device__ __forceinline__ ItemPlanes item_planes(const float2* const* planes, const Items& it) {
    ItemPlanes ip;
#pragma unroll
    for (int k = 0; k < kPfItems; ++k) ip.p[k] = planes[k < it.n ? it.dp[k] >> 16 : 0];
    // redefine the pointers here, after their loads completed: otherwise the
    // wait for them is placed at their first use inside the row loop, where
    // it is repeated every row and waits for the stores and loads in flight
#pragma unroll
    for (int k = 0; k < kPfItems; ++k) asm volatile("" : "+v"(ip.p[k]));
    return ip;
}

// Converts a pixel pair {re0, im0, re1, im1} into its 16-byte record and
// stores it in ring slot `slot`.
template <bool SPLIT>
__device__ __forceinline__ void store_unit(const CohArgs& a, void* lds, uint32_t dp, int slot, f32x4 z) {
    const int d = (int)(dp >> 16), px = (int)(dp & 0xffffu);
    u32x4* rec = reinterpret_cast<u32x4*>(lds) + d * a.plane + slot * a.pitch + px;
    u32x4 v;
    if constexpr (SPLIT) {
        typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
        typedef float f32x2 __attribute__((ext_vector_type(2)));
        const f32x2 re = {z[0], z[2]}, im = {z[1], z[3]};
        const bf16x2 rh = __builtin_convertvector(re, bf16x2);  // round to nearest even
        const bf16x2 ih = __builtin_convertvector(im, bf16x2);
        const bf16x2 rl = __builtin_convertvector(re - __builtin_convertvector(rh, f32x2), bf16x2);
        const bf16x2 il = __builtin_convertvector(im - __builtin_convertvector(ih, f32x2), bf16x2);
        v[0] = __builtin_bit_cast(uint32_t, rh);
        v[1] = __builtin_bit_cast(uint32_t, rl);
        v[2] = __builtin_bit_cast(uint32_t, ih);
        v[3] = __builtin_bit_cast(uint32_t, il);
    } else {
        v = __builtin_bit_cast(u32x4, z);
    }
    *rec = v;
}

__device__ __forceinline__ int next_slot(int s, int wy) { return s + 1 == wy ? 0 : s + 1; }

// Start the global loads of the prefetched units of the next kPfRows rows;
// they complete while the current row's pixels are computed.  Every slot is
// loaded, at row and column indices clamped into the image (two 8-byte loads
// per unit), with no branch: the number of loads in flight is then the same
// on every path, so a later wait for a load issued before them (the first
// pixel's mask) can leave them in flight.  Out-of-image entries are zeroed
// at commit time (fix_unit), slots beyond the thread's items or the rows
// the next output row needs are never committed.
__device__ __forceinline__ f32x4 fetch_clamped(const CohArgs& a, const float2* plane, uint32_t dp, int64_t y,
                                               int64_t x0) {
    const Geometry& g = a.g;
    const int64_t x = x0 + 2 * (int)(dp & 0xffffu);
    const int64_t yc = y < 0 ? 0 : (y >= g.R ? g.R - 1 : y);
    const int64_t xa = x < 0 ? 0 : (x >= g.C ? g.C - 1 : x);
    const int64_t xb = x + 1 < 0 ? 0 : (x + 1 >= g.C ? g.C - 1 : x + 1);
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(1))) const f32x2 gf32x2;
    gf32x2* row = (gf32x2*)plane + yc * g.C;
    const f32x2 u = row[xa], v = row[xb];
    return f32x4{u[0], u[1], v[0], v[1]};
}

// Zeroes the entries of a clamped unit that lie outside the image.
__device__ __forceinline__ f32x4 fix_unit(const CohArgs& a, uint32_t dp, int64_t y, int64_t x0, f32x4 z) {
    const Geometry& g = a.g;
    const int64_t x = x0 + 2 * (int)(dp & 0xffffu);
    const bool yin = y >= 0 && y < g.R;
    const bool in0 = yin && x >= 0 && x < g.C, in1 = yin && x + 1 >= 0 && x + 1 < g.C;
    return f32x4{in0 ? z[0] : 0.f, in0 ? z[1] : 0.f, in1 ? z[2] : 0.f, in1 ? z[3] : 0.f};
}

template <int NT>
__device__ __forceinline__ void prefetch_rows(const CohArgs& a, const ItemPlanes& ip, const Items& it,
                                              RowLoad<NT>& pf, int64_t y_first, int64_t x0) {
#pragma unroll
    for (int r = 0; r < kPfRows<NT>; ++r)
#pragma unroll
        for (int k = 0; k < kPfItems; ++k) pf.v[r][k] = fetch_clamped(a, ip.p[k], it.dp[k], y_first + r, x0);
}

template <int NT, bool SPLIT>
__device__ __forceinline__ void commit_rows(const CohArgs& a, const float2* const* planes, const Items& it,
                                            void* lds, const RowLoad<NT>& pf, int64_t y_first, int nrows,
                                            int64_t x0) {
    const int s0 = ring_slot(y_first, a.g.wy);
    int slot = s0;
#pragma unroll
    for (int r = 0; r < kPfRows<NT>; ++r) {
        if (r < nrows) {
#pragma unroll
            for (int k = 0; k < kPfItems; ++k)
                if (k < it.n) store_unit<SPLIT>(a, lds, it.dp[k], slot, fix_unit(a, it.dp[k], y_first + r, x0, pf.v[r][k]));
            slot = next_slot(slot, a.g.wy);
        }
    }
    // units outside the prefetch grid
    slot = s0;
    for (int r = 0; r < nrows; ++r) {
#pragma unroll
        for (int k = 0; k < kMaxItems; ++k)
            if (k < it.n && (k >= kPfItems || r >= kPfRows<NT>))
                store_unit<SPLIT>(a, lds, it.dp[k], slot, fetch_unit(a, planes, it.dp[k], y_first + r, x0));
        slot = next_slot(slot, a.g.wy);
    }
}

// List the window pairs of output pixel (oy, ox) that hold an SHP as entries
// of two words: the record offset inside an image plane and a mask word
// (SPLIT: 0xffff per selected BF16 half; FP32: bit 0 / bit 1 for the first /
// second pixel).  The list is padded with zero entries to a multiple of
// `ppk`.  `mw` holds mask word `lane` of the pixel (lanes < nw); `s0` is the
// ring slot of the window's first row.  Returns the padded count (uniform
// over the wave).
template <bool SPLIT>
__device__ __forceinline__ int build_pairs(const CohArgs& a, uint32_t* table, int64_t ox, int64_t x0, int s0,
                           uint32_t mw, int ppk, int lane) {
    const Geometry& g = a.g;
    const int64_t cx = ox * g.sx + g.sx / 2;
    const int rel = (int)(cx - g.hx - x0);  // >= 0 by construction of x0
    const int rec0 = rel >> 1, par = rel & 1;
    const int ppr = g.hx + 1;  // pairs per window row
    int n = 0;
    for (int base = 0; base < a.n_pairs; base += 64) {
        const int j = base + lane;
        const int dy = fast_div(j, a.inv_ppr), px = j - dy * ppr;
        const int dx0 = 2 * px - par;
        const int b0 = dy * g.wx + dx0;
        // bits b0 and b0 + 1 of the window mask (pairs never straddle rows)
        const uint32_t w0 = __shfl(mw, (b0 >= 0 ? b0 : 0) >> 5, 64);
        const uint32_t w1 = __shfl(mw, (b0 + 1) >> 5, 64);
        uint32_t bits = 0;
        if (j < a.n_pairs) {
            if (dx0 >= 0) bits |= (w0 >> (b0 & 31)) & 1u;
            if (dx0 + 1 <= 2 * g.hx) bits |= ((w1 >> ((b0 + 1) & 31)) & 1u) << 1;
        }
        int slot = s0 + dy;
        slot -= slot >= g.wy ? g.wy : 0;
        const bool keep = bits != 0;
        const uint64_t bal = __ballot(keep);
        const int before = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0));
        if (keep) {
            uint32_t mword = bits;
            if constexpr (SPLIT) mword = ((bits & 1u) ? 0x0000ffffu : 0u) | ((bits & 2u) ? 0xffff0000u : 0u);
            table[2 * (n + before)] = (uint32_t)(slot * a.pitch + rec0 + px);
            table[2 * (n + before) + 1] = mword;
        }
        n += __popcll(bal);
    }
    const int npad = (n + ppk - 1) / ppk * ppk;
    for (int j = n + lane; j < npad; j += 64) {
        table[2 * j] = 0u;
        table[2 * j + 1] = 0u;
    }
    return npad;
}

template <int NT>
__device__ __forceinline__ void transpose_read(float* S, const typename Acc<NT>::T& x,
                                               typename Acc<NT>::T& xt, int lane) {
    constexpr int LD = NT + 1;
    const int j = lane & (NT - 1);
#pragma unroll
    for (int v = 0; v < Acc<NT>::R; ++v) S[Acc<NT>::row(lane, v) * LD + j] = x[v];
    wave_sync();
#pragma unroll
    for (int v = 0; v < Acc<NT>::R; ++v) xt[v] = S[j * LD + Acc<NT>::row(lane, v)];
    wave_sync();
}

// Marks R loaded values as used here (R a multiple of 4): loads whose values
// are only used under a per-entry condition can be moved into one branch
// each, where each waits for its data before the next is issued; placed
// after a run of loads, this keeps them back to back with one wait.
template <int R>
__device__ __forceinline__ void keep_loaded(float (&v)[R]) {
#pragma unroll
    for (int k = 0; k < R; k += 4) asm volatile("" : "+v"(v[k]), "+v"(v[k + 1]), "+v"(v[k + 2]), "+v"(v[k + 3]));
}

// Normalise and store one pixel's matrix from Re/Im in accumulator layout.
template <int NT, bool SPLIT>
__device__ __forceinline__ void store_pixel(const CohArgs& a, float* S, const typename Acc<NT>::T& re,
                            const typename Acc<NT>::T& im, int64_t pix, int lane) {
    constexpr int LD = NT + 1;
    // the transpose-free split path keeps only the diagonal in the wave's scratch
    float* diag = S + (SPLIT && NT == 32 ? 0 : NT * LD);
    const int j = lane & (NT - 1);
    const int N = a.N;
#pragma unroll
    for (int v = 0; v < Acc<NT>::R; ++v)
        if (Acc<NT>::row(lane, v) == j) diag[j] = re[v];
    wave_sync();
    const float dj = diag[j];
    const bool bad = (j < N) && !(dj > 0.f && dj <= 3.4e38f);
    const bool invalid = __ballot(bad) != 0;
    // hardware reciprocal square roots (about 1 ulp), far inside the coherence tolerance
    const float isj = __builtin_amdgcn_rsqf(dj);
    if (a.diag && lane < NT && j < N) a.diag[pix * N + j] = dj;
    const int packed = a.packed;
    float2* out = a.coh + pix * (int64_t)(packed ? (N * (N + 1)) >> 1 : N * N);
    if (invalid) {  // uniform: some image without power over the SHPs, or a non-finite sum
#pragma unroll
        for (int v = 0; v < Acc<NT>::R; ++v) {
            const int i = Acc<NT>::row(lane, v);
            if (i < N && j < N && (!packed || i <= j))
                out[packed ? ((i * (2 * N - i - 1)) >> 1) + j : i * N + j] =
                    make_float2(__builtin_nanf(""), __builtin_nanf(""));
        }
        wave_sync();
        return;
    }
    // each row's reciprocal square root is formed once (by the lanes of its
    // column) and shared through the diagonal scratch
    wave_sync();  // every lane has read its diagonal entry
    diag[j] = isj;
    wave_sync();
    float si[Acc<NT>::R];  // 1 / sqrt of the diagonal entries of this lane's rows (row < NT)
#pragma unroll
    for (int v = 0; v < Acc<NT>::R; ++v) si[v] = diag[Acc<NT>::row(lane, v)];
    keep_loaded(si);
#pragma unroll
    for (int v = 0; v < Acc<NT>::R; ++v) {
        const int i = Acc<NT>::row(lane, v);
        if (i < N && j < N && (!packed || i <= j)) {
            const float isi = si[v];
            float2 c = make_float2(re[v] * isi * isj, im[v] * isi * isj);
            if (i == j) c = make_float2(1.f, 0.f);
            // packed: entry (i, j >= i) of the row-major upper triangle
            out[packed ? ((i * (2 * N - i - 1)) >> 1) + j : i * N + j] = c;
        }
    }
    wave_sync();
}

template <int NT, bool SPLIT>
__device__ __forceinline__ void pixel_gram(const CohArgs& a, const void* lds, const uint32_t* table, int npad,
                           int lane, typename Acc<NT>::T& re, typename Acc<NT>::T& im, float* S) {
    typedef typename Acc<NT>::T AT;
    const int d = lane & (NT - 1);
    const bool live = d < a.N;
    const int g = lane / NT;  // k-group of this lane
    // Dead rows (image index >= N) read a valid plane and are masked to zero
    // on both operand sides; their columns are never stored.
    const int dd = live ? d : a.N - 1;
    const uint32_t live_mask = live ? 0xffffffffu : 0u;
    AT whh = {}, v1 = {};
    if constexpr (SPLIT && NT == 32) {
        // 32-row tiles: both triangles of Re A and Im A straight from the
        // MFMAs, so no transpose (and no transpose scratch in LDS):
        //   Re A = sum s (rh rh + rh rl + rl rh + ih ih + ih il + il ih)
        //   Im A = sum s (ih rh + ih rl + il rh) - sum s (rh ih + rh il + rl ih)
        // with the SHP bit on both operands of every product.
        AT re1 = {}, imn = {};
        constexpr int PPK = 8;  // pairs per k-step
        const u32x4* P = reinterpret_cast<const u32x4*>(lds) + dd * a.plane;
        const u32x4* E = reinterpret_cast<const u32x4*>(table) + 2 * g;  // 4 entries per group
        u32x4 e01 = E[0], e23 = E[1];
        for (int ks = 0; ks < npad; ks += PPK) {
            const u32x4 q0 = P[e01[0]], q1 = P[e01[2]], q2 = P[e23[0]], q3 = P[e23[2]];
            u32x4 n01 = e01, n23 = e23;
            if (ks + PPK < npad) {
                n01 = E[(ks + PPK) / 2];
                n23 = E[(ks + PPK) / 2 + 1];
            }
            const uint32_t m0 = e01[1] & live_mask, m1 = e01[3] & live_mask;
            const uint32_t m2 = e23[1] & live_mask, m3 = e23[3] & live_mask;
            // Both operands masked: s in {0, 1}, so (s x_m)(s x_n) = s x_m x_n
            // exactly, and the masked words go straight into the operand
            // registers (no unmasked copies are assembled).
            const u32x4 rhm = {q0[0] & m0, q1[0] & m1, q2[0] & m2, q3[0] & m3};
            const u32x4 rlm = {q0[1] & m0, q1[1] & m1, q2[1] & m2, q3[1] & m3};
            const u32x4 ihm = {q0[2] & m0, q1[2] & m1, q2[2] & m2, q3[2] & m3};
            const u32x4 ilm = {q0[3] & m0, q1[3] & m1, q2[3] & m2, q3[3] & m3};
            const bf16x8 Rhm = __builtin_bit_cast(bf16x8, rhm), Rlm = __builtin_bit_cast(bf16x8, rlm);
            const bf16x8 Ihm = __builtin_bit_cast(bf16x8, ihm), Ilm = __builtin_bit_cast(bf16x8, ilm);
            // four accumulation chains, interleaved
            whh = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Rhm, Rhm, whh, 0, 0, 0);
            v1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ihm, Rhm, v1, 0, 0, 0);
            re1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Rhm, Rlm, re1, 0, 0, 0);
            imn = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Rhm, Ihm, imn, 0, 0, 0);
            whh = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Rlm, Rhm, whh, 0, 0, 0);
            v1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ihm, Rlm, v1, 0, 0, 0);
            re1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ihm, Ihm, re1, 0, 0, 0);
            imn = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Rhm, Ilm, imn, 0, 0, 0);
            whh = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ihm, Ilm, whh, 0, 0, 0);
            v1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ilm, Rhm, v1, 0, 0, 0);
            re1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ilm, Ihm, re1, 0, 0, 0);
            imn = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Rlm, Ihm, imn, 0, 0, 0);
            e01 = n01;
            e23 = n23;
        }
        (void)S;
        re = whh + re1;
        im = v1 - imn;
    } else if constexpr (SPLIT) {
        AT whl = {}, v2 = {};
        constexpr int PPK = NT == 16 ? 16 : 8;  // pairs per k-step
        const u32x4* P = reinterpret_cast<const u32x4*>(lds) + dd * a.plane;
        const u32x4* E = reinterpret_cast<const u32x4*>(table) + 2 * g;  // 4 entries per group
        // the entries of the next k-step are read one step ahead
        u32x4 e01 = E[0], e23 = E[1];
        for (int ks = 0; ks < npad; ks += PPK) {
            const u32x4 q0 = P[e01[0]], q1 = P[e01[2]], q2 = P[e23[0]], q3 = P[e23[2]];
            u32x4 n01 = e01, n23 = e23;
            if (ks + PPK < npad) {
                n01 = E[(ks + PPK) / 2];
                n23 = E[(ks + PPK) / 2 + 1];
            }
            const uint32_t m0 = e01[1] & live_mask, m1 = e01[3] & live_mask;
            const uint32_t m2 = e23[1] & live_mask, m3 = e23[3] & live_mask;
            // both operands masked (s x_m)(s x_n) = s x_m x_n, s in {0, 1}: the
            // masked words go straight into the operand registers
            const u32x4 rhm = {q0[0] & m0, q1[0] & m1, q2[0] & m2, q3[0] & m3};
            const u32x4 rlm = {q0[1] & m0, q1[1] & m1, q2[1] & m2, q3[1] & m3};
            const u32x4 ihm = {q0[2] & m0, q1[2] & m1, q2[2] & m2, q3[2] & m3};
            const u32x4 ilm = {q0[3] & m0, q1[3] & m1, q2[3] & m2, q3[3] & m3};
            const bf16x8 Rh = __builtin_bit_cast(bf16x8, rhm), Rl = __builtin_bit_cast(bf16x8, rlm);
            const bf16x8 Ih = __builtin_bit_cast(bf16x8, ihm), Il = __builtin_bit_cast(bf16x8, ilm);
            const bf16x8 Rm = Rh, Im = Ih;
            // the four accumulation chains are interleaved so that no MFMA
            // waits on the one just issued
            if constexpr (NT == 16) {
                whh = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Rm, Rh, whh, 0, 0, 0);
                whl = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Rm, Rl, whl, 0, 0, 0);
                v1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Rm, Ih, v1, 0, 0, 0);
                v2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Im, Rl, v2, 0, 0, 0);
                whh = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Im, Ih, whh, 0, 0, 0);
                whl = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Im, Il, whl, 0, 0, 0);
                v1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Rm, Il, v1, 0, 0, 0);
            } else {
                whh = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Rm, Rh, whh, 0, 0, 0);
                whl = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Rm, Rl, whl, 0, 0, 0);
                v1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Rm, Ih, v1, 0, 0, 0);
                v2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Im, Rl, v2, 0, 0, 0);
                whh = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Im, Ih, whh, 0, 0, 0);
                whl = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Im, Il, whl, 0, 0, 0);
                v1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Rm, Il, v1, 0, 0, 0);
            }
            e01 = n01;
            e23 = n23;
        }
        AT t;
        transpose_read<NT>(S, whl, t, lane);
        re = whh + whl + t;
        const AT u = v2 - v1;
        transpose_read<NT>(S, u, t, lane);
        im = u - t;
    } else {
        constexpr int SPK = NT == 16 ? 4 : 2;  // samples per k-step
        typedef float f32x2 __attribute__((ext_vector_type(2)));
        typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
        constexpr int STEP = SPK / 2;  // pairs per k-step
        constexpr int U = 8;           // k-steps per batch
        const f32x2* P = reinterpret_cast<const f32x2*>(lds) + 2 * dd * a.plane;
        const int half = g & 1;
        const int eoff = g >> 1;  // which pair of the k-step (16x16x4 only)
        // Each sample needs two dependent LDS reads (its list entry, then the
        // record): a batch of U k-steps issues its U entry reads, then its U
        // sample reads, then its MFMAs in the plain k-step order, so two LDS
        // round trips serve U k-steps.  Reads past the end of the list are
        // clamped to its last step and their products skipped.
        const u32x2* T = reinterpret_cast<const u32x2*>(table) + eoff;
        const int lastc = npad > STEP ? npad - STEP : 0;
        for (int ks = 0; ks < npad; ks += U * STEP) {
            u32x2 e[U];
            f32x2 z[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = ks + u * STEP;
                e[u] = T[k < lastc ? k : lastc];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) z[u] = P[2 * e[u][0] + half];  // {re, im} of this lane's sample
            // the reads are used here, before the first product: otherwise
            // the compiler sinks each into its k-step's branch below, which
            // serialises them again
#pragma unroll
            for (int u = 0; u < U; ++u) asm volatile("" ::"v"(z[u]), "v"(e[u][1]));
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (ks + u * STEP >= npad) break;  // uniform
                const bool on = live && ((e[u][1] >> half) & 1u);
                const float r = z[u][0], im_ = z[u][1];
                const float rm = on ? r : 0.f, imm = on ? im_ : 0.f;
                // the SHP bit on both operands: (s x_m)(s x_n) = s x_m x_n, and a
                // non-finite sample outside the SHPs (sharing a record with one)
                // contributes an exact zero instead of 0 * NaN
                if constexpr (NT == 16) {
                    whh = __builtin_amdgcn_mfma_f32_16x16x4f32(rm, rm, whh, 0, 0, 0);
                    v1 = __builtin_amdgcn_mfma_f32_16x16x4f32(rm, imm, v1, 0, 0, 0);
                    whh = __builtin_amdgcn_mfma_f32_16x16x4f32(imm, imm, whh, 0, 0, 0);
                } else {
                    whh = __builtin_amdgcn_mfma_f32_32x32x2f32(rm, rm, whh, 0, 0, 0);
                    v1 = __builtin_amdgcn_mfma_f32_32x32x2f32(rm, imm, v1, 0, 0, 0);
                    whh = __builtin_amdgcn_mfma_f32_32x32x2f32(imm, imm, whh, 0, 0, 0);
                }
            }
        }
        re = whh;
        AT t;
        transpose_read<NT>(S, v1, t, lane);
        im = t - v1;
    }
}

template <int NT, bool SPLIT>
__device__ __forceinline__ void coherence_body(const CohArgs& a, const float2* const* planes, int64_t strip, int64_t band,
                               uint32_t* lds_words) {
    const Geometry& g = a.g;
    const int nthreads = blockDim.x;
    const int nwaves = nthreads >> 6;
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    const int64_t ox0 = strip * a.TXo;
    const int64_t ox1 = ox0 + a.TXo < g.oC ? ox0 + a.TXo : g.oC;
    const int64_t oy0 = a.oy_lo + band * a.rows_per_wg;
    const int64_t oy1 = oy0 + a.rows_per_wg < a.oy_hi ? oy0 + a.rows_per_wg : a.oy_hi;
    const int64_t x0 = (ox0 * g.sx + g.sx / 2 - g.hx) & ~(int64_t)1;
    const int data_words = 4 * a.N * a.plane;  // one 16-byte record per pixel pair
    uint32_t* wave_area = lds_words + data_words + wave * a.wave_words;
    float* S = reinterpret_cast<float*>(wave_area);
    constexpr int PPK = SPLIT ? (NT == 16 ? 16 : 8) : (NT == 16 ? 2 : 1);

    // ring slot of the first window row of output row oy
    auto first_slot = [&](int64_t oy) {
        int s0 = (int)((oy * g.sy + g.sy / 2 - g.hy) % g.wy);
        return s0 + (s0 < 0 ? g.wy : 0);
    };
    RowLoad<NT> pf;
    const Items items = make_items(a, nthreads);
    const ItemPlanes iplanes = item_planes(planes, items);
    // prologue: the full window of the first output row, kPfRows rows per
    // batch of loads (the same values in the same ring slots as row by row)
    {
        const int64_t yw = oy0 * g.sy + g.sy / 2 - g.hy;
        for (int r0 = 0; r0 < g.wy; r0 += kPfRows<NT>) {
            const int nr = g.wy - r0 < kPfRows<NT> ? g.wy - r0 : kPfRows<NT>;
            prefetch_rows<NT>(a, iplanes, items, pf, yw + r0, x0);
            commit_rows<NT, SPLIT>(a, planes, items, lds_words, pf, yw + r0, nr, x0);
        }
    }
    __syncthreads();
    for (int64_t oy = oy0; oy < oy1; ++oy) {
        const int64_t cy = oy * g.sy + g.sy / 2;
        // rows the next output row needs that are not staged yet
        const int64_t next_first = (cy + g.hy + 1) > (cy + g.sy - g.hy) ? (cy + g.hy + 1) : (cy + g.sy - g.hy);
        const int next_rows = (int)((cy + g.sy + g.hy) - next_first + 1);
        const bool more = oy + 1 < oy1;
        // The first pixel's mask is requested before the row prefetch and
        // waited for right after it is issued: loads complete in order, so
        // that wait leaves the prefetch in flight.  Each value is redefined
        // once its load has arrived (an empty asm), so that no wait for the
        // prefetch is merged into the paths that follow.
        int64_t ox = ox0 + wave;
        uint32_t mfirst = 0;
        if (ox < ox1 && lane < g.nw) mfirst = a.mask[(oy * g.oC + ox) * g.nw + lane];
        prefetch_rows<NT>(a, iplanes, items, pf, next_first, x0);  // unused after the last row
        asm volatile("" : "+v"(mfirst));
        const int s0 = first_slot(oy);
        for (; ox < ox1; ox += nwaves) {
            uint32_t mw = mfirst;
            if (ox != ox0 + wave) {  // later pixels of a strip wider than the wave count
                uint32_t m = lane < g.nw ? a.mask[(oy * g.oC + ox) * g.nw + lane] : 0u;
                asm volatile("" : "+v"(m));
                mw = m;
            }
            const int npad = build_pairs<SPLIT>(a, wave_area, ox, x0, s0, mw, PPK, lane);
            wave_sync();
            typename Acc<NT>::T re, im;
            pixel_gram<NT, SPLIT>(a, lds_words, wave_area, npad, lane, re, im, S);
            store_pixel<NT, SPLIT>(a, S, re, im, (oy - a.oy_lo) * g.oC + ox, lane);
        }
        __syncthreads();  // every wave is done with the rows about to be replaced
        if (more) {
            commit_rows<NT, SPLIT>(a, planes, items, lds_words, pf, next_first, next_rows, x0);
            __syncthreads();
        }
    }
}

}  // namespace
}  // namespace plk
