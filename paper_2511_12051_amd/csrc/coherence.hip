// Windowed sample coherence over SHPs (paper eq. sample-coherence) on the
// matrix cores.
//
// For one output pixel let r_m(k), i_m(k) be the real and imaginary parts of
// image m at its k-th window sample and s(k) in {0,1} its SHP bit.  Then
//   Re A = sum_k s (r r^T + i i^T),  Im A = S^T - S,  S = sum_k s r i^T,
// three real Gram-type products X diag(s) Y^T whose rows are the images
// (at most 16 or 32) and whose reduction runs over window samples - exactly
// the operand shape of an MFMA, with A- and B-fragments read by the same
// lane.  The SHP weight is applied by zeroing masked samples of both
// operands (s in {0, 1}, so (s x_m)(s x_n) = s x_m x_n exactly, and a
// non-finite sample outside the SHPs adds an exact zero).
//
// Plain FP32: v_mfma_f32_{16x16x4,32x32x2}f32 on r, i directly.
// Split BF16: each value x = hi + lo with hi = bf16(x), lo = bf16(x - hi)
// (about 16 significant bits).  Products hi*hi + hi*lo + lo*hi are kept, lo*lo
// dropped:  Re A = Whh + Whl + Whl^T  with Whl = sum s (r_h r_l^T + i_h i_l^T),
// S = V1 + V2^T with V1 = sum s r_h (i_h + i_l)^T, V2 = sum s i_h r_l^T, so
// Im A = U - U^T with U = V2 - V1;  seven v_mfma_f32_{16x16x32,32x32x16}_bf16
// per k-step.  32-row tiles keep all six products of each of Re A and Im A
// (twelve MFMAs per k-step) instead of forming the transposed terms through
// LDS, which frees the transpose scratch for a wider strip of the ring.
//
// Data movement: a workgroup owns a strip of TXo output columns and walks
// down a band of output rows.  The window rows it needs live in an LDS ring
// of (2*half_y+1) input rows, one plane per image, so that the 16 or 32
// lanes of one fragment read 16 or 32 different planes at one offset (the
// plane stride is 4 mod 64 words: the lanes of a group hit distinct banks).
// Moving to the next output row loads only the stride_y new input rows.  The
// plane stores 16-byte records of two horizontally adjacent pixels starting
// at an even column: {re_hi, re_lo, im_hi, im_lo} as BF16 pairs, or
// {re, im, re, im} in FP32.  Every window is cut into such pairs; per pixel a
// wavefront first lists the pairs that hold at least one SHP (record offset
// and a mask word), then runs the MFMA loop over that compacted list with one
// 16-byte LDS read per pair.
#include <cmath>

#include "batch_device.hpp"
#include "coherence_device.hpp"
#include "internal.hpp"

namespace plk {
namespace {

template <int NT, bool SPLIT>
__global__ __launch_bounds__(64 * kWaves<NT>) void coherence_kernel(CohArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds_words[];
    coherence_body<NT, SPLIT>(a, a.t.p, blockIdx.x, blockIdx.y, lds_words);
}

template <int NT, bool SPLIT>
__global__ __launch_bounds__(64 * kWaves<NT>) void coherence_batch(BatchRange<CohArgs> r) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds_words[];
    for (int64_t b = blockIdx.x; b < r.total; b += gridDim.x) {
        const int k = batch_item(r.starts, r.n, b);
        // a local copy of the arguments: the body then keeps them in registers
        // instead of re-loading them from the table after each store; its
        // plane pointers are read from the table itself
        const CohArgs a = r.items[k];
        const int64_t local = b - r.starts[k];
        // the body ends with a workgroup barrier, after which LDS may be refilled
        coherence_body<NT, SPLIT>(a, r.items[k].t.p, local % a.n_strips, local / a.n_strips, lds_words);
    }
}

template <int NT, bool SPLIT>
const void* kernel_of(bool batch) {
    return batch ? reinterpret_cast<const void*>(coherence_batch<NT, SPLIT>)
                 : reinterpret_cast<const void*>(coherence_kernel<NT, SPLIT>);
}

const void* coherence_fn(int nt, bool split, bool batch) {
    if (nt == 16) return split ? kernel_of<16, true>(batch) : kernel_of<16, false>(batch);
    return split ? kernel_of<32, true>(batch) : kernel_of<32, false>(batch);
}

// compute units of the current device (queried once per device)
int device_cus() {
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (!cus[dev]) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1) c = 1;
        cus[dev] = c;
    }
    return cus[dev];
}

}  // namespace

size_t coherence_args(CohArgs* ap, int nt, bool split, int txo_max, int rows_req, int64_t* blocks) {
    CohArgs& a = *ap;
    const Geometry& g = a.g;
    const size_t lds_cap = max_lds_bytes();
    const int PPK = split ? (nt == 16 ? 16 : 8) : (nt == 16 ? 2 : 1);
    // transpose scratch and diagonal; the split 32-row path transposes nothing
    const int scratch_words = (split && nt == 32) ? nt : nt * (nt + 1) + nt;
    const int table_words = ((2 * (a.n_pairs + PPK) + 3) / 4) * 4;
    a.wave_words = ((scratch_words > table_words ? scratch_words : table_words) + 3) / 4 * 4;
    int chosen = 0;
    size_t lds = 0;
    for (int txo = txo_max < 16 ? txo_max : 16; txo >= 1; --txo) {
        int tile_w = (txo - 1) * g.sx + 2 * g.hx + 3;
        tile_w += tile_w & 1;
        const int pitch = tile_w >> 1;
        int plane = g.wy * pitch;
        plane += (1 - plane % 16 + 16) % 16;  // records = 1 mod 16: stride 4 mod 64 words
        const size_t bytes = (size_t)16 * a.N * plane + (size_t)waves_of(nt) * a.wave_words * 4;
        if (bytes <= lds_cap) {
            chosen = txo;
            a.tile_w = tile_w;
            a.pitch = pitch;
            a.plane = plane;
            lds = bytes;
            break;
        }
    }
    if (!chosen) return 0;
    a.TXo = chosen;
    a.inv_ppr = 1.0f / (float)(g.hx + 1);
    if ((int64_t)a.N * (a.tile_w >> 1) > (int64_t)kMaxItems * 64 * waves_of(nt)) return 0;
    a.vec_rows = (g.C % 2) == 0;
    for (int d = 0; d < a.N; ++d)
        if (reinterpret_cast<uintptr_t>(a.t.p[d]) & 15) a.vec_rows = 0;
    a.n_strips = (g.oC + chosen - 1) / chosen;
    int64_t rows = rows_req;
    const int64_t nrows = a.oy_hi - a.oy_lo;
    if (rows <= 0) {  // enough workgroups to fill the chip several times over
        rows = (nrows * a.n_strips + 2047) / 2048;
        if (rows < 4) rows = 4;
        // Each CU holds lds_cap / lds workgroups at a time, so the grid runs in
        // rounds of that many per CU; a last round that is nearly empty still
        // costs about one workgroup's duration.  Among band counts near this
        // one, take the one that best fills the last round, weighed against
        // the prologue of each band (its first wy - sy rows, loaded three rows
        // per batch, so about a third of the cost of as many computed rows)
        const int64_t slots = (int64_t)device_cus() * (int64_t)(lds_cap / lds > 0 ? lds_cap / lds : 1);
        const int64_t nb0 = (nrows + rows - 1) / rows;
        if (a.n_strips * nb0 >= 4 * slots) {
            double best = -1.0;
            int64_t best_rows = rows;
            for (int64_t nb = (nb0 + 1) / 2; nb <= 3 * nb0 && nb <= nrows; ++nb) {
                const int64_t r = (nrows + nb - 1) / nb;
                const double rounds = (double)(a.n_strips * ((nrows + r - 1) / r)) / (double)slots;
                const double fill = rounds / std::ceil(rounds);
                const double pro = (double)(g.wy > g.sy ? g.wy - g.sy : 0) / (3.0 * (double)r * g.sy);
                const double score = fill / (1.0 + pro);
                if (score > best + 1e-9) {
                    best = score;
                    best_rows = r;
                }
            }
            rows = best_rows;
        }
    }
    if (rows > nrows) rows = nrows;
    a.rows_per_wg = (int)rows;
    *blocks = a.n_strips * ((nrows + rows - 1) / rows);
    return lds;
}

pl_status launch_coherence(const PlaneTable& t, int N, const Geometry& g, const uint32_t* mask,
                           int prec, float2* coh, float* diag, hipStream_t s) {
    CohArgs a{};
    a.diag = diag;
    a.t = t;
    a.N = N;
    a.g = g;
    a.mask = mask;
    a.coh = coh;
    a.packed = 0;
    a.oy_lo = 0;
    a.oy_hi = g.oR;
    return launch_coherence_args(a, prec, s);
}

pl_status launch_coherence_rows(const PlaneTable& t, int N, const Geometry& g, const uint32_t* mask,
                                int prec, float2* coh, int packed, int64_t oy_lo, int64_t oy_hi,
                                hipStream_t s) {
    CohArgs a{};
    a.diag = nullptr;
    a.t = t;
    a.N = N;
    a.g = g;
    a.mask = mask;
    a.coh = coh;
    a.packed = packed;
    a.oy_lo = oy_lo;
    a.oy_hi = oy_hi;
    return launch_coherence_args(a, prec, s);
}

pl_status launch_coherence_args(CohArgs& a, int prec, hipStream_t s) {
    const Geometry& g = a.g;
    const int N = a.N;
    a.n_pairs = g.wy * (g.hx + 1);
    const bool split = prec == PL_PREC_SPLIT_BF16;
    const int nt = N <= 16 ? 16 : 32;
    int64_t blocks = 0;
    const size_t lds = coherence_args(&a, nt, split, coherence_strip(nt), 0, &blocks);
    if (!lds) return fail(PL_ERR_UNSUPPORTED, "pl_estimate_coherence: window too large for LDS");
    const int64_t n_bands = blocks / a.n_strips;
    if (a.n_strips > 2147483647LL || n_bands > 65535)
        return fail(PL_ERR_UNSUPPORTED, "pl_estimate_coherence: output grid too large");
    const void* fn = coherence_fn(nt, split, false);
    pl_status st = allow_dynamic_lds(fn, lds);
    if (st != PL_OK) return st;
    // always the full wave count: the staging layout (and its size check) assumes it
    const int nwaves = waves_of(nt);
    if (nt == 16) {
        if (split) hipLaunchKernelGGL((coherence_kernel<16, true>), dim3((unsigned)a.n_strips, (unsigned)n_bands), dim3(64 * nwaves), lds, s, a);
        else hipLaunchKernelGGL((coherence_kernel<16, false>), dim3((unsigned)a.n_strips, (unsigned)n_bands), dim3(64 * nwaves), lds, s, a);
    } else {
        if (split) hipLaunchKernelGGL((coherence_kernel<32, true>), dim3((unsigned)a.n_strips, (unsigned)n_bands), dim3(64 * nwaves), lds, s, a);
        else hipLaunchKernelGGL((coherence_kernel<32, false>), dim3((unsigned)a.n_strips, (unsigned)n_bands), dim3(64 * nwaves), lds, s, a);
    }
    return launch_ok("coherence kernel");
}

const void* coherence_batch_fn(int nt, bool split) { return coherence_fn(nt, split, true); }

int coherence_threads(int nt) { return 64 * waves_of(nt); }
int coherence_strip(int nt) { return nt == 16 ? 12 : 8; }  // one output column per wavefront and row

// the caller has raised the kernel's dynamic LDS limit (allow_dynamic_lds)
pl_status launch_coherence_batch(const BatchRange<CohArgs>& r, int nt, bool split, size_t lds, int64_t grid,
                                 hipStream_t s) {
    if (r.total == 0) return PL_OK;
    const dim3 gr((unsigned)grid), bl(64 * waves_of(nt));
    if (nt == 16) {
        if (split) hipLaunchKernelGGL((coherence_batch<16, true>), gr, bl, lds, s, r);
        else hipLaunchKernelGGL((coherence_batch<16, false>), gr, bl, lds, s, r);
    } else {
        if (split) hipLaunchKernelGGL((coherence_batch<32, true>), gr, bl, lds, s, r);
        else hipLaunchKernelGGL((coherence_batch<32, false>), gr, bl, lds, s, r);
    }
    return launch_ok("batched coherence kernel");
}

}  // namespace plk
