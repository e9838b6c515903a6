// Sequential estimator: the mini-stack reference scheme of the paper's
// Sec. 2.2 (Fig. 1).  Host-side state machine over the kernels; device state
// is the ring of the K_max most recent compressed SLCs and the ring of the
// K_max + 1 most recent per-mini-stack amplitude statistics (the ancillary
// products stored with each compressed SLC, Sec. 3.1).
#include <cmath>
#include <cstring>
#include <new>

#include "internal.hpp"

using namespace plk;

struct pl_seq {
    pl_seq_params p;
    Geometry g;
    int64_t plane = 0, opix = 0;
    int64_t count = 0;  // mini-stacks pushed
    float2* kappa = nullptr;  // [K_max][R][C] ring
    double* means = nullptr;  // [K_max+1][R][C] ring
    double* vars = nullptr;
    double* mean_m = nullptr;  // merged statistics
    double* var_m = nullptr;
    uint32_t* mask = nullptr;
    uint16_t* cnt = nullptr;
    float2* coh = nullptr;      // [opix][N][N], N = M + K_max
    float2* phasors = nullptr;  // [N][opix]
    uint8_t* flags = nullptr;   // [opix]
    void* owned = nullptr;      // the device block, when the driver allocated it
};

namespace {

constexpr uint64_t kMagic = 0x706c696e6b736571ull;  // "plinkseq"

struct CkptHeader {
    uint64_t magic;
    int64_t R, C;
    int32_t M, K_max;
    pl_window w;
    int64_t count;
    int32_t reference, pad;
    double weight_decay;
};

// Device state in one block: each array starts on a 256-byte boundary.  With
// base == nullptr only the size is computed.
size_t carve(pl_seq* s, unsigned char* base) {
    const pl_seq_params& p = s->p;
    const int N = p.M + p.K_max;
    size_t off = 0;
    auto take = [&]<class T>(T** ptr, size_t n) {
        off = (off + 255) & ~(size_t)255;
        *ptr = base && n ? reinterpret_cast<T*>(base + off) : nullptr;
        off += n * sizeof(T);
    };
    take(&s->kappa, (size_t)p.K_max * s->plane);
    take(&s->means, (size_t)(p.K_max + 1) * s->plane);
    take(&s->vars, (size_t)(p.K_max + 1) * s->plane);
    take(&s->mean_m, (size_t)s->plane);
    take(&s->var_m, (size_t)s->plane);
    take(&s->mask, (size_t)s->opix * s->g.nw);
    take(&s->cnt, (size_t)s->opix);
    take(&s->coh, (size_t)s->opix * N * N);
    take(&s->phasors, (size_t)s->opix * N);
    take(&s->flags, (size_t)s->opix);
    return (off + 255) & ~(size_t)255;
}

void release(pl_seq* s) {
    if (s->owned) (void)hipFree(s->owned);
    s->owned = nullptr;
}

// checks the parameters and fills the host part of the driver
pl_status setup(const pl_seq_params* params, pl_seq* s, const char* fn) {
    const pl_seq_params& p = *params;
    Geometry g;
    if (!make_geometry(p.R, p.C, p.w, &g) || g.oR < 1 || g.oC < 1)
        return fail(PL_ERR_SHAPE, "%s: bad image size or window", fn);
    if (p.M < 1 || p.K_max < 0 || p.M + p.K_max > kMaxN)
        return fail(PL_ERR_UNSUPPORTED, "%s: need 1 <= M and M + K_max <= %d", fn, kMaxN);
    if (!(p.alpha > 0 && p.alpha < 1)) return fail(PL_ERR_INVALID_ARG, "%s: alpha outside (0,1)", fn);
    if (p.precision != PL_PREC_FP32 && p.precision != PL_PREC_SPLIT_BF16)
        return fail(PL_ERR_INVALID_ARG, "%s: unknown precision", fn);
    if (p.method != PL_LINK_EMI && p.method != PL_LINK_EVD) return fail(PL_ERR_INVALID_ARG, "%s: unknown method", fn);
    if (p.reference != PL_SEQ_REF_COMPRESSED && p.reference != PL_SEQ_REF_LAST)
        return fail(PL_ERR_INVALID_ARG, "%s: unknown reference mode", fn);
    if (!(p.weight_decay > 0 && p.weight_decay <= 1))
        return fail(PL_ERR_INVALID_ARG, "%s: weight_decay outside (0, 1]", fn);
    s->p = p;
    s->g = g;
    s->plane = p.R * p.C;
    s->opix = g.oR * g.oC;
    return PL_OK;
}

size_t state_bytes(const pl_seq* s) {
    return sizeof(CkptHeader) + (size_t)s->p.K_max * s->plane * sizeof(float2) +
           (size_t)2 * (s->p.K_max + 1) * s->plane * sizeof(double);
}

}  // namespace

extern "C" {

pl_status pl_seq_workspace_size(const pl_seq_params* params, size_t* bytes) {
    if (!params || !bytes) return fail(PL_ERR_INVALID_ARG, "pl_seq_workspace_size: NULL pointer");
    pl_seq s;
    const pl_status st = setup(params, &s, "pl_seq_workspace_size");
    if (st != PL_OK) return st;
    *bytes = carve(&s, nullptr);
    return PL_OK;
}

pl_status pl_seq_create_in(const pl_seq_params* params, void* dev_workspace, size_t bytes, pl_seq** out) {
    if (!params || !out || !dev_workspace) return fail(PL_ERR_INVALID_ARG, "pl_seq_create_in: NULL pointer");
    if (reinterpret_cast<uintptr_t>(dev_workspace) & 255)
        return fail(PL_ERR_INVALID_ARG, "pl_seq_create_in: workspace not 256-byte aligned");
    pl_seq* s = new (std::nothrow) pl_seq();
    if (!s) return fail(PL_ERR_WORKSPACE, "pl_seq_create_in: out of host memory");
    pl_status st = setup(params, s, "pl_seq_create_in");
    if (st == PL_OK && bytes < carve(s, nullptr))
        st = fail(PL_ERR_WORKSPACE, "pl_seq_create_in: workspace of %zu bytes, the driver needs %zu", bytes,
                  carve(s, nullptr));
    if (st != PL_OK) {
        delete s;
        return st;
    }
    carve(s, static_cast<unsigned char*>(dev_workspace));
    *out = s;
    return PL_OK;
}

pl_status pl_seq_create(const pl_seq_params* params, pl_seq** out) {
    if (!params || !out) return fail(PL_ERR_INVALID_ARG, "pl_seq_create: NULL pointer");
    pl_seq* s = new (std::nothrow) pl_seq();
    if (!s) return fail(PL_ERR_WORKSPACE, "pl_seq_create: out of host memory");
    pl_status st = setup(params, s, "pl_seq_create");
    if (st == PL_OK) st = hip_ok(hipMalloc(&s->owned, carve(s, nullptr)), "pl_seq_create: device state");
    if (st != PL_OK) {
        release(s);
        delete s;
        return st;
    }
    carve(s, static_cast<unsigned char*>(s->owned));
    *out = s;
    return PL_OK;
}

pl_status pl_seq_destroy(pl_seq* s) {
    if (!s) return PL_OK;
    release(s);
    delete s;
    return PL_OK;
}

pl_status pl_seq_count(const pl_seq* s, int64_t* count) {
    if (!s || !count) return fail(PL_ERR_INVALID_ARG, "pl_seq_count: NULL pointer");
    *count = s->count;
    return PL_OK;
}

pl_status pl_seq_push(pl_seq* s, const pl_c64* new_slcs, pl_c64* phasors_out, pl_c64* kappa_out,
                      uint8_t* flags_out, uint64_t* counters, pl_stream stream) {
    if (!s || !new_slcs || !phasors_out) return fail(PL_ERR_INVALID_ARG, "pl_seq_push: NULL pointer");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(counters);
    const pl_seq_params& p = s->p;
    const int64_t k = s->count;
    const int M = p.M, Kmax = p.K_max;
    const int K = (int)(k < Kmax ? k : Kmax);  // compressed SLCs in this mini-stack
    const int N = K + M;
    const int64_t plane = s->plane;
    const float2* znew = reinterpret_cast<const float2*>(new_slcs);

    // amplitude statistics of the new images into the statistics ring
    const int slot = (int)(k % (Kmax + 1));
    PlaneTable tn = contiguous_planes(new_slcs, M, plane);
    pl_status r = launch_amp_stats(tn, 0, M, plane, s->means + slot * plane, s->vars + slot * plane, st);
    if (r != PL_OK) return r;
    // merge the statistics of mini-stacks k-K..k, weights M decay^age
    const double* mp[64];
    const double* vp[64];
    double w[64];
    const int G = K + 1;
    double n_eff = 0.0;
    for (int j = 0; j < G; ++j) {
        const int sl = (int)((k - K + j) % (Kmax + 1));
        mp[j] = s->means + sl * plane;
        vp[j] = s->vars + sl * plane;
        w[j] = (double)M * std::pow(p.weight_decay, (double)(G - 1 - j));
        n_eff += w[j];
    }
    r = launch_merge_stats(mp, vp, w, G, plane, s->mean_m, s->var_m, st);
    if (r != PL_OK) return r;
    r = launch_shp_select(s->mean_m, s->var_m, s->g, n_eff, p.alpha, s->mask, s->cnt, cnt, st);
    if (r != PL_OK) return r;
    // stack = [kappa_{k-K} .. kappa_{k-1} | new], no copies
    PlaneTable t{};
    for (int j = 0; j < K; ++j) t.p[j] = s->kappa + ((k - K + j) % Kmax) * plane;
    for (int j = 0; j < M; ++j) t.p[K + j] = znew + j * plane;
    r = launch_coherence(t, N, s->g, s->mask, p.precision, s->coh, nullptr, st);
    if (r != PL_OK) return r;
    const int ref = K > 0 ? K - 1 : 0;  // the most recent compressed SLC
    r = launch_phase_link(link_args(s->coh, N, s->opix, ref, p.method, s->phasors, nullptr, nullptr, s->flags, cnt),
                          st);
    if (r != PL_OK) return r;
    // new compressed SLC over the real images; it replaces the oldest ring
    // entry, which the kernels above have already consumed (stream order)
    float2* knew = Kmax > 0 ? s->kappa + (k % Kmax) * plane : reinterpret_cast<float2*>(kappa_out);
    if (knew) {
        // PL_SEQ_REF_LAST: phasors re-referenced to the last real image,
        // kappa = sum conj(zeta_i conj(zeta_last)) z_i = zeta_last kappa
        r = launch_compress(t, N, K, s->g, s->phasors, knew, st, p.reference == PL_SEQ_REF_LAST ? N - 1 : -1);
        if (r != PL_OK) return r;
    }
    r = hip_ok(hipMemcpyAsync(phasors_out, s->phasors + (int64_t)K * s->opix,
                              (size_t)M * s->opix * sizeof(float2), hipMemcpyDeviceToDevice, st),
               "pl_seq_push: phasor copy");
    if (r != PL_OK) return r;
    if (kappa_out && Kmax > 0) {
        r = hip_ok(hipMemcpyAsync(kappa_out, knew, (size_t)plane * sizeof(float2), hipMemcpyDeviceToDevice, st),
                   "pl_seq_push: kappa copy");
        if (r != PL_OK) return r;
    }
    if (flags_out) {
        r = hip_ok(hipMemcpyAsync(flags_out, s->flags, (size_t)s->opix, hipMemcpyDeviceToDevice, st),
                   "pl_seq_push: flag copy");
        if (r != PL_OK) return r;
    }
    s->count = k + 1;
    return PL_OK;
}

pl_status pl_seq_last_mask(const pl_seq* s, uint32_t* mask, pl_stream stream) {
    if (!s || !mask) return fail(PL_ERR_INVALID_ARG, "pl_seq_last_mask: NULL pointer");
    if (s->count == 0) return fail(PL_ERR_STATE, "pl_seq_last_mask: no mini-stack pushed yet");
    return hip_ok(hipMemcpyAsync(mask, s->mask, (size_t)s->opix * s->g.nw * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                                 reinterpret_cast<hipStream_t>(stream)),
                  "pl_seq_last_mask: copy");
}

pl_status pl_seq_state_size(const pl_seq* s, size_t* bytes) {
    if (!s || !bytes) return fail(PL_ERR_INVALID_ARG, "pl_seq_state_size: NULL pointer");
    *bytes = state_bytes(s);
    return PL_OK;
}

pl_status pl_seq_save(const pl_seq* s, void* host_buf, size_t bytes, pl_stream stream) {
    if (!s || !host_buf) return fail(PL_ERR_INVALID_ARG, "pl_seq_save: NULL pointer");
    if (bytes < state_bytes(s)) return fail(PL_ERR_WORKSPACE, "pl_seq_save: buffer too small");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    CkptHeader h{kMagic, s->p.R, s->p.C, s->p.M, s->p.K_max, s->p.w, s->count, s->p.reference, 0,
                 s->p.weight_decay};
    unsigned char* b = static_cast<unsigned char*>(host_buf);
    std::memcpy(b, &h, sizeof h);
    size_t off = sizeof h;
    const size_t kb = (size_t)s->p.K_max * s->plane * sizeof(float2);
    const size_t sb = (size_t)(s->p.K_max + 1) * s->plane * sizeof(double);
    pl_status r = PL_OK;
    if (kb) r = hip_ok(hipMemcpyAsync(b + off, s->kappa, kb, hipMemcpyDeviceToHost, st), "pl_seq_save");
    off += kb;
    if (r == PL_OK) r = hip_ok(hipMemcpyAsync(b + off, s->means, sb, hipMemcpyDeviceToHost, st), "pl_seq_save");
    off += sb;
    if (r == PL_OK) r = hip_ok(hipMemcpyAsync(b + off, s->vars, sb, hipMemcpyDeviceToHost, st), "pl_seq_save");
    if (r == PL_OK) r = hip_ok(hipStreamSynchronize(st), "pl_seq_save: synchronize");
    return r;
}

pl_status pl_seq_load(pl_seq* s, const void* host_buf, size_t bytes, pl_stream stream) {
    if (!s || !host_buf) return fail(PL_ERR_INVALID_ARG, "pl_seq_load: NULL pointer");
    if (bytes < state_bytes(s)) return fail(PL_ERR_WORKSPACE, "pl_seq_load: buffer too small");
    CkptHeader h;
    const unsigned char* b = static_cast<const unsigned char*>(host_buf);
    std::memcpy(&h, b, sizeof h);
    if (h.magic != kMagic || h.R != s->p.R || h.C != s->p.C || h.M != s->p.M || h.K_max != s->p.K_max ||
        std::memcmp(&h.w, &s->p.w, sizeof h.w) != 0 || h.count < 0 || h.reference != s->p.reference ||
        h.weight_decay != s->p.weight_decay)
        return fail(PL_ERR_STATE, "pl_seq_load: checkpoint does not match this driver");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    size_t off = sizeof h;
    const size_t kb = (size_t)s->p.K_max * s->plane * sizeof(float2);
    const size_t sb = (size_t)(s->p.K_max + 1) * s->plane * sizeof(double);
    pl_status r = PL_OK;
    if (kb) r = hip_ok(hipMemcpyAsync(s->kappa, b + off, kb, hipMemcpyHostToDevice, st), "pl_seq_load");
    off += kb;
    if (r == PL_OK) r = hip_ok(hipMemcpyAsync(s->means, b + off, sb, hipMemcpyHostToDevice, st), "pl_seq_load");
    off += sb;
    if (r == PL_OK) r = hip_ok(hipMemcpyAsync(s->vars, b + off, sb, hipMemcpyHostToDevice, st), "pl_seq_load");
    if (r == PL_OK) r = hip_ok(hipStreamSynchronize(st), "pl_seq_load: synchronize");
    if (r == PL_OK) s->count = h.count;
    return r;
}

}  // extern "C"
