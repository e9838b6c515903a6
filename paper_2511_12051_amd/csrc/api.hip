// Host side of the C ABI: argument checks, error strings, dispatch.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "internal.hpp"

namespace plk {

static thread_local char g_last_error[512] = "";

pl_status fail(pl_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return s;
}

pl_status hip_ok(hipError_t e, const char* what) {
    if (e == hipSuccess) return PL_OK;
    return fail(PL_ERR_HIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

pl_status launch_ok(const char* what) { return hip_ok(hipGetLastError(), what); }

bool make_geometry(int64_t R, int64_t C, pl_window w, Geometry* g) {
    if (R <= 0 || C <= 0) return false;
    if (w.half_x < 0 || w.half_y < 0 || w.stride_x < 1 || w.stride_y < 1) return false;
    int64_t wx = 2 * (int64_t)w.half_x + 1, wy = 2 * (int64_t)w.half_y + 1;
    if (wx * wy > PL_MAX_WINDOW) return false;
    g->R = R;
    g->C = C;
    g->hx = w.half_x;
    g->hy = w.half_y;
    g->sx = w.stride_x;
    g->sy = w.stride_y;
    g->wx = (int)wx;
    g->wy = (int)wy;
    g->W = (int)(wx * wy);
    g->nw = (g->W + 31) / 32;
    g->oR = R / w.stride_y;
    g->oC = C / w.stride_x;
    return true;
}

PlaneTable contiguous_planes(const pl_c64* stack, int N, int64_t plane) {
    PlaneTable t{};
    for (int i = 0; i < N && i < kMaxN; ++i)
        t.p[i] = reinterpret_cast<const float2*>(stack) + (int64_t)i * plane;
    return t;
}

size_t max_lds_bytes() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 65536;
    return v > 0 ? (size_t)v : 65536;
}

pl_status allow_dynamic_lds(const void* fn, size_t lds) {
    if (lds <= 65536) return PL_OK;
    return hip_ok(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                  "dynamic LDS attribute");
}

}  // namespace plk

using namespace plk;

static hipStream_t S(pl_stream s) { return reinterpret_cast<hipStream_t>(s); }

#define PL_CHECK(cond, status, ...) \
    do {                            \
        if (!(cond)) return fail(status, __VA_ARGS__); \
    } while (0)

// ---- fused coherence + linking over bands of output rows
static size_t fused_row_bytes(int N, const Geometry& g) {
    return (size_t)g.oC * (size_t)(N * (N + 1) / 2) * sizeof(float2);
}

namespace plk {
namespace {
// the checked body shared by the fused entry points: rows per band from the
// buffer size, then per band one coherence launch into the buffer and one
// linking launch out of it (stream order separates the bands)
pl_status fused_run(const pl_c64* stack, int32_t N, const Geometry& g, const uint32_t* mask, pl_precision prec,
                    int32_t ref_idx, pl_link_method method, pl_c64* phasors, float* phase, float* lambda,
                    float* temp_coh, uint8_t* flags, uint64_t* counters, float2* buf, size_t buf_bytes,
                    hipStream_t s) {
    const size_t row = fused_row_bytes(N, g);
    int64_t rows = (int64_t)(buf_bytes / row);
    if (rows > g.oR) rows = g.oR;
    const int64_t P = g.oR * g.oC;
    PlaneTable t = contiguous_planes(stack, N, g.R * g.C);
    for (int64_t a = 0; a < g.oR; a += rows) {
        const int64_t b = a + rows < g.oR ? a + rows : g.oR;
        pl_status r = launch_coherence_rows(t, N, g, mask, (int)prec, buf, 1, a, b, s);
        if (r != PL_OK) return r;
        const int64_t off = a * g.oC;
        LinkArgs la = link_args(buf, N, (b - a) * g.oC, ref_idx, (int)method,
                                reinterpret_cast<float2*>(phasors) + off, phase ? phase + off : nullptr,
                                lambda ? lambda + off : nullptr, flags ? flags + off : nullptr,
                                reinterpret_cast<unsigned long long*>(counters));
        la.tcoh = temp_coh ? temp_coh + off : nullptr;
        la.packed = 1;
        la.ostride = P;
        r = launch_phase_link(la, s);
        if (r != PL_OK) return r;
    }
    return PL_OK;
}

pl_status fused_check(const pl_c64* stack, int32_t N, int64_t R, int64_t C, pl_window w, const uint32_t* mask,
                      pl_precision prec, int32_t ref_idx, pl_link_method method, const pl_c64* phasors,
                      const char* who, Geometry* g) {
    PL_CHECK(stack && mask && phasors, PL_ERR_INVALID_ARG, "%s: NULL pointer", who);
    PL_CHECK(N >= 1 && N <= kMaxN, PL_ERR_UNSUPPORTED, "%s: N=%d outside 1..%d", who, N, kMaxN);
    PL_CHECK(make_geometry(R, C, w, g), PL_ERR_SHAPE, "%s: bad image size or window", who);
    PL_CHECK(g->oR >= 1 && g->oC >= 1, PL_ERR_SHAPE, "%s: image smaller than one stride", who);
    PL_CHECK(ref_idx >= 0 && ref_idx < N, PL_ERR_INVALID_ARG, "%s: ref_idx %d outside 0..%d", who, ref_idx, N - 1);
    PL_CHECK(prec == PL_PREC_FP32 || prec == PL_PREC_SPLIT_BF16, PL_ERR_INVALID_ARG, "%s: unknown precision %d",
             who, (int)prec);
    PL_CHECK(method == PL_LINK_EMI || method == PL_LINK_EVD, PL_ERR_INVALID_ARG, "%s: unknown method %d", who,
             (int)method);
    return PL_OK;
}
}  // namespace
}  // namespace plk

// ---- the fused path without allocation: the band buffer is a file-scope
// device array, one copy per GPU, whose device address is looked up once per
// device (the array's name in host code is not a device address)
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace plk {
namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

pl_status scratch_address(void** out) {
    int dev = 0;
    pl_status r = hip_ok(hipGetDevice(&dev), "pl_phase_link_fused_noalloc: current device");
    if (r != PL_OK) return r;
    if (dev < 0 || dev >= 64) return fail(PL_ERR_UNSUPPORTED, "pl_phase_link_fused_noalloc: device %d", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        r = hip_ok(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "pl_phase_link_fused_noalloc: scratch address");
        if (r != PL_OK) return r;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return PL_OK;
}
}  // namespace
}  // namespace plk


extern "C" {

const char* pl_version(void) { return "plink 0.1 (gfx950)"; }

const char* pl_status_string(pl_status s) {
    switch (s) {
        case PL_OK: return "ok";
        case PL_ERR_INVALID_ARG: return "invalid argument";
        case PL_ERR_SHAPE: return "inconsistent shape";
        case PL_ERR_UNSUPPORTED: return "unsupported";
        case PL_ERR_HIP: return "HIP error";
        case PL_ERR_WORKSPACE: return "buffer too small";
        case PL_ERR_STATE: return "state mismatch";
    }
    return "unknown status";
}

const char* pl_last_error(void) { return g_last_error; }

pl_status pl_output_grid(int64_t R, int64_t C, pl_window w, int64_t* oR, int64_t* oC) {
    Geometry g;
    PL_CHECK(oR && oC, PL_ERR_INVALID_ARG, "pl_output_grid: NULL output");
    PL_CHECK(make_geometry(R, C, w, &g), PL_ERR_SHAPE, "pl_output_grid: bad image size or window");
    *oR = g.oR;
    *oC = g.oC;
    return PL_OK;
}

int32_t pl_mask_words(pl_window w) {
    Geometry g;
    if (!make_geometry(1, 1, w, &g)) return 0;
    return g.nw;
}

pl_status pl_amplitude_stats(const pl_c64* slc, int32_t M, int64_t R, int64_t C, double* mean,
                             double* var, pl_stream stream) {
    PL_CHECK(slc && mean && var, PL_ERR_INVALID_ARG, "pl_amplitude_stats: NULL pointer");
    PL_CHECK(M >= 1 && M <= kMaxN, PL_ERR_UNSUPPORTED, "pl_amplitude_stats: M=%d outside 1..%d", M, kMaxN);
    PL_CHECK(R >= 1 && C >= 1, PL_ERR_SHAPE, "pl_amplitude_stats: empty image");
    PlaneTable t = contiguous_planes(slc, M, R * C);
    return launch_amp_stats(t, 0, M, R * C, mean, var, S(stream));
}

pl_status pl_merge_amplitude_stats(const double* means, const double* vars, const double* weights,
                                   int32_t G, int64_t R, int64_t C, double* mean_out,
                                   double* var_out, pl_stream stream) {
    PL_CHECK(means && vars && weights && mean_out && var_out, PL_ERR_INVALID_ARG,
             "pl_merge_amplitude_stats: NULL pointer");
    PL_CHECK(G >= 1 && G <= 64, PL_ERR_UNSUPPORTED, "pl_merge_amplitude_stats: G=%d outside 1..64", G);
    PL_CHECK(R >= 1 && C >= 1, PL_ERR_SHAPE, "pl_merge_amplitude_stats: empty image");
    for (int i = 0; i < G; ++i)
        PL_CHECK(weights[i] > 0 && std::isfinite(weights[i]), PL_ERR_INVALID_ARG,
                 "pl_merge_amplitude_stats: weight %d not positive", i);
    const double* mp[64];
    const double* vp[64];
    for (int i = 0; i < G; ++i) {
        mp[i] = means + (int64_t)i * R * C;
        vp[i] = vars + (int64_t)i * R * C;
    }
    return launch_merge_stats(mp, vp, weights, G, R * C, mean_out, var_out, S(stream));
}

pl_status pl_shp_select(const double* mean, const double* var, int64_t R, int64_t C, double n_eff,
                        pl_window w, double alpha, uint32_t* mask, uint16_t* count,
                        uint64_t* counters, pl_stream stream) {
    Geometry g;
    PL_CHECK(mean && var && mask && count, PL_ERR_INVALID_ARG, "pl_shp_select: NULL pointer");
    PL_CHECK(make_geometry(R, C, w, &g), PL_ERR_SHAPE, "pl_shp_select: bad image size or window");
    PL_CHECK(g.oR >= 1 && g.oC >= 1, PL_ERR_SHAPE, "pl_shp_select: image smaller than one stride");
    PL_CHECK(n_eff > 0 && std::isfinite(n_eff), PL_ERR_INVALID_ARG, "pl_shp_select: n_eff must be > 0");
    PL_CHECK(alpha > 0 && alpha < 1, PL_ERR_INVALID_ARG, "pl_shp_select: alpha must lie in (0, 1)");
    return launch_shp_select(mean, var, g, n_eff, alpha, mask, count,
                             reinterpret_cast<unsigned long long*>(counters), S(stream));
}

pl_status pl_estimate_coherence(const pl_c64* stack, int32_t N, int64_t R, int64_t C, pl_window w,
                                const uint32_t* mask, pl_precision prec, pl_c64* coh,
                                pl_stream stream) {
    Geometry g;
    PL_CHECK(stack && mask && coh, PL_ERR_INVALID_ARG, "pl_estimate_coherence: NULL pointer");
    PL_CHECK(N >= 1 && N <= kMaxN, PL_ERR_UNSUPPORTED, "pl_estimate_coherence: N=%d outside 1..%d", N, kMaxN);
    PL_CHECK(make_geometry(R, C, w, &g), PL_ERR_SHAPE, "pl_estimate_coherence: bad image size or window");
    PL_CHECK(g.oR >= 1 && g.oC >= 1, PL_ERR_SHAPE, "pl_estimate_coherence: image smaller than one stride");
    PL_CHECK(prec == PL_PREC_FP32 || prec == PL_PREC_SPLIT_BF16, PL_ERR_INVALID_ARG,
             "pl_estimate_coherence: unknown precision %d", (int)prec);
    PlaneTable t = contiguous_planes(stack, N, R * C);
    return launch_coherence(t, N, g, mask, (int)prec, reinterpret_cast<float2*>(coh), nullptr, S(stream));
}

pl_status pl_sync_report(pl_stream stream, const uint64_t* counters, pl_report* out) {
    PL_CHECK(counters && out, PL_ERR_INVALID_ARG, "pl_sync_report: NULL pointer");
    uint64_t h[PL_NUM_COUNTERS];
    pl_status r = hip_ok(hipStreamSynchronize(S(stream)), "pl_sync_report: synchronize");
    if (r != PL_OK) return r;
    r = hip_ok(hipMemcpy(h, counters, sizeof h, hipMemcpyDeviceToHost), "pl_sync_report: copy");
    if (r != PL_OK) return r;
    out->glrt_band = (int64_t)h[PL_CNT_GLRT_BAND];
    out->glrt_recheck = (int64_t)h[PL_CNT_GLRT_RECHECK];
    out->evd_fallbacks = (int64_t)h[PL_CNT_EVD];
    out->invalid = (int64_t)h[PL_CNT_INVALID];
    out->not_converged = (int64_t)h[PL_CNT_NOT_CONVERGED];
    out->shift_retries = (int64_t)h[PL_CNT_SHIFT_RETRY];
    out->iterations = (int64_t)h[PL_CNT_ITERS];
    for (int b = 0; b < 16; ++b) out->iter_hist[b] = (int64_t)h[PL_CNT_ITER_HIST + b];
    return PL_OK;
}

pl_status pl_phase_link(const pl_c64* coh, int32_t N, int64_t npix, int32_t ref_idx,
                        pl_link_method method, pl_c64* phasors, float* phase, float* lambda,
                        float* temp_coh, uint8_t* flags, uint64_t* counters, pl_stream stream) {
    PL_CHECK(N >= 1 && N <= kMaxN, PL_ERR_UNSUPPORTED, "pl_phase_link: N=%d outside 1..%d", N, kMaxN);
    PL_CHECK(npix >= 0, PL_ERR_SHAPE, "pl_phase_link: negative pixel count");
    PL_CHECK(npix == 0 || (coh && phasors), PL_ERR_INVALID_ARG, "pl_phase_link: NULL pointer");
    PL_CHECK(ref_idx >= 0 && ref_idx < N, PL_ERR_INVALID_ARG, "pl_phase_link: ref_idx %d outside 0..%d",
             ref_idx, N - 1);
    PL_CHECK(method == PL_LINK_EMI || method == PL_LINK_EVD, PL_ERR_INVALID_ARG,
             "pl_phase_link: unknown method %d", (int)method);
    if (npix == 0) return PL_OK;
    LinkArgs a = link_args(reinterpret_cast<const float2*>(coh), N, npix, ref_idx, (int)method,
                           reinterpret_cast<float2*>(phasors), phase, lambda, flags,
                           reinterpret_cast<unsigned long long*>(counters));
    a.tcoh = temp_coh;
    return launch_phase_link(a, S(stream));
}

pl_status pl_phase_link_fused_workspace(int32_t N, int64_t R, int64_t C, pl_window w, size_t* min_bytes,
                                        size_t* all_rows_bytes) {
    Geometry g;
    PL_CHECK(min_bytes || all_rows_bytes, PL_ERR_INVALID_ARG, "pl_phase_link_fused_workspace: NULL output");
    PL_CHECK(N >= 1 && N <= kMaxN, PL_ERR_UNSUPPORTED, "pl_phase_link_fused_workspace: N=%d outside 1..%d", N, kMaxN);
    PL_CHECK(make_geometry(R, C, w, &g), PL_ERR_SHAPE, "pl_phase_link_fused_workspace: bad image size or window");
    PL_CHECK(g.oR >= 1 && g.oC >= 1, PL_ERR_SHAPE, "pl_phase_link_fused_workspace: image smaller than one stride");
    if (min_bytes) *min_bytes = fused_row_bytes(N, g);
    if (all_rows_bytes) *all_rows_bytes = fused_row_bytes(N, g) * (size_t)g.oR;
    return PL_OK;
}


pl_status pl_phase_link_fused_noalloc(const pl_c64* stack, int32_t N, int64_t R, int64_t C, pl_window w,
                                      const uint32_t* mask, pl_precision prec, int32_t ref_idx,
                                      pl_link_method method, pl_c64* phasors, float* phase, float* lambda,
                                      float* temp_coh, uint8_t* flags, uint64_t* counters, pl_stream stream) {
    Geometry g;
    pl_status r =
        fused_check(stack, N, R, C, w, mask, prec, ref_idx, method, phasors, "pl_phase_link_fused_noalloc", &g);
    if (r != PL_OK) return r;
    PL_CHECK(fused_row_bytes(N, g) <= kScratchBytes, PL_ERR_WORKSPACE,
             "pl_phase_link_fused_noalloc: one output row needs %zu bytes of the %zu-byte scratch buffer",
             fused_row_bytes(N, g), kScratchBytes);
    void* ptr = nullptr;
    r = scratch_address(&ptr);
    if (r != PL_OK) return r;
    return fused_run(stack, N, g, mask, prec, ref_idx, method, phasors, phase, lambda, temp_coh, flags, counters,
                     static_cast<float2*>(ptr), kScratchBytes, S(stream));
}

pl_status pl_phase_link_fused(const pl_c64* stack, int32_t N, int64_t R, int64_t C, pl_window w,
                              const uint32_t* mask, pl_precision prec, int32_t ref_idx,
                              pl_link_method method, pl_c64* phasors, float* phase, float* lambda,
                              float* temp_coh, uint8_t* flags, uint64_t* counters, void* workspace,
                              size_t ws_bytes, pl_stream stream) {
    Geometry g;
    pl_status r = fused_check(stack, N, R, C, w, mask, prec, ref_idx, method, phasors, "pl_phase_link_fused", &g);
    if (r != PL_OK) return r;
    PL_CHECK(workspace, PL_ERR_INVALID_ARG, "pl_phase_link_fused: NULL workspace");
    PL_CHECK(ws_bytes >= fused_row_bytes(N, g), PL_ERR_WORKSPACE,
             "pl_phase_link_fused: workspace of %zu bytes, one output row needs %zu", ws_bytes, fused_row_bytes(N, g));
    return fused_run(stack, N, g, mask, prec, ref_idx, method, phasors, phase, lambda, temp_coh, flags, counters,
                     static_cast<float2*>(workspace), ws_bytes, S(stream));
}

// workspace of the adjoint: C [P][N][N] c64 | diag(A) [P][N] f32 |
// S [N(N+1)/2][P] c64, each 256-byte aligned
static size_t vjp_layout(int N, int64_t P, size_t* off_diag, size_t* off_s) {
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t coh = up((size_t)P * N * N * 8);
    const size_t diag = up((size_t)P * N * 4);
    const size_t sb = up((size_t)P * (N * (N + 1) / 2) * 8);
    if (off_diag) *off_diag = coh;
    if (off_s) *off_s = coh + diag;
    return coh + diag + sb;
}

pl_status pl_phase_link_vjp_workspace(int32_t N, int64_t R, int64_t C, pl_window w, size_t* bytes) {
    Geometry g;
    PL_CHECK(bytes, PL_ERR_INVALID_ARG, "pl_phase_link_vjp_workspace: NULL output");
    PL_CHECK(N >= 1 && N <= kMaxN, PL_ERR_UNSUPPORTED, "pl_phase_link_vjp_workspace: N=%d outside 1..%d", N, kMaxN);
    PL_CHECK(make_geometry(R, C, w, &g), PL_ERR_SHAPE, "pl_phase_link_vjp_workspace: bad image size or window");
    PL_CHECK(g.oR >= 1 && g.oC >= 1, PL_ERR_SHAPE, "pl_phase_link_vjp_workspace: image smaller than one stride");
    *bytes = vjp_layout(N, g.oR * g.oC, nullptr, nullptr);
    return PL_OK;
}

pl_status pl_phase_link_vjp(const pl_c64* stack, int32_t N, int64_t R, int64_t C, pl_window w,
                            const uint32_t* mask, const uint8_t* flags, int32_t ref_idx,
                            pl_precision prec, const float* grad_phase, pl_c64* grad_stack,
                            void* workspace, size_t ws_bytes, pl_stream stream) {
    Geometry g;
    PL_CHECK(stack && mask && flags && grad_phase && grad_stack && workspace, PL_ERR_INVALID_ARG,
             "pl_phase_link_vjp: NULL pointer");
    PL_CHECK(N >= 1 && N <= kMaxN, PL_ERR_UNSUPPORTED, "pl_phase_link_vjp: N=%d outside 1..%d", N, kMaxN);
    PL_CHECK(make_geometry(R, C, w, &g), PL_ERR_SHAPE, "pl_phase_link_vjp: bad image size or window");
    PL_CHECK(g.oR >= 1 && g.oC >= 1, PL_ERR_SHAPE, "pl_phase_link_vjp: image smaller than one stride");
    PL_CHECK(ref_idx >= 0 && ref_idx < N, PL_ERR_INVALID_ARG, "pl_phase_link_vjp: ref_idx %d outside 0..%d",
             ref_idx, N - 1);
    PL_CHECK(prec == PL_PREC_FP32 || prec == PL_PREC_SPLIT_BF16, PL_ERR_INVALID_ARG,
             "pl_phase_link_vjp: unknown precision %d", (int)prec);
    const int64_t P = g.oR * g.oC;
    size_t off_diag = 0, off_s = 0;
    const size_t need = vjp_layout(N, P, &off_diag, &off_s);
    PL_CHECK(ws_bytes >= need, PL_ERR_WORKSPACE, "pl_phase_link_vjp: workspace of %zu bytes, %zu needed",
             ws_bytes, need);
    unsigned char* ws = static_cast<unsigned char*>(workspace);
    float2* coh = reinterpret_cast<float2*>(ws);
    float* diag = reinterpret_cast<float*>(ws + off_diag);
    float2* Sm = reinterpret_cast<float2*>(ws + off_s);
    PlaneTable t = contiguous_planes(stack, N, R * C);
    pl_status r = launch_coherence(t, N, g, mask, (int)prec, coh, diag, S(stream));
    if (r != PL_OK) return r;
    r = launch_link_vjp(coh, diag, flags, grad_phase, N, P, ref_idx, Sm, S(stream));
    if (r != PL_OK) return r;
    return launch_vjp_gather(t, N, g, mask, Sm, reinterpret_cast<float2*>(grad_stack), S(stream));
}

pl_status pl_compress_ministack(const pl_c64* stack, int32_t N, int32_t first_real, int64_t R,
                                int64_t C, pl_window w, const pl_c64* phasors, pl_c64* kappa,
                                pl_stream stream) {
    Geometry g;
    PL_CHECK(stack && phasors && kappa, PL_ERR_INVALID_ARG, "pl_compress_ministack: NULL pointer");
    PL_CHECK(N >= 1 && N <= kMaxN, PL_ERR_UNSUPPORTED, "pl_compress_ministack: N=%d outside 1..%d", N, kMaxN);
    PL_CHECK(first_real >= 0 && first_real < N, PL_ERR_INVALID_ARG,
             "pl_compress_ministack: first_real %d outside 0..%d", first_real, N - 1);
    PL_CHECK(make_geometry(R, C, w, &g), PL_ERR_SHAPE, "pl_compress_ministack: bad image size or window");
    PL_CHECK(g.oR >= 1 && g.oC >= 1, PL_ERR_SHAPE, "pl_compress_ministack: image smaller than one stride");
    PlaneTable t = contiguous_planes(stack, N, R * C);
    return launch_compress(t, N, first_real, g, reinterpret_cast<const float2*>(phasors),
                           reinterpret_cast<float2*>(kappa), S(stream));
}

}  // extern "C"
