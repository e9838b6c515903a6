// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "plink.h"

namespace plk {

constexpr int kMaxN = PL_MAX_N;

// Device addresses of the images of a stack.  Images need not be contiguous,
// so the sequential driver links [compressed | new] without copying.
struct PlaneTable {
    const float2* p[kMaxN];
};

// Window and output-grid geometry of one call.
struct Geometry {
    int64_t R, C, oR, oC;
    int hx, hy, sx, sy;  // half-window and stride (x = columns, y = rows)
    int wx, wy, W, nw;   // window width/height, window size, mask words
};

bool make_geometry(int64_t R, int64_t C, pl_window w, Geometry* g);

// error reporting (thread-local message, returned status)
pl_status fail(pl_status s, const char* fmt, ...);
pl_status hip_ok(hipError_t e, const char* what);
pl_status launch_ok(const char* what);

PlaneTable contiguous_planes(const pl_c64* stack, int N, int64_t plane);

// LDS bytes one workgroup may use on the current device.
size_t max_lds_bytes();

// ---- kernel launchers (each validates nothing; callers check arguments)
pl_status launch_amp_stats(const PlaneTable& t, int first, int M, int64_t npix, double* mean,
                           double* var, hipStream_t s);
pl_status launch_merge_stats(const double* const* means, const double* const* vars,
                             const double* weights, int G, int64_t npix, double* mean_out,
                             double* var_out, hipStream_t s);
pl_status launch_shp_select(const double* mean, const double* var, const Geometry& g,
                            double n_eff, double alpha, uint32_t* mask, uint16_t* count,
                            unsigned long long* counters, hipStream_t s);
// diag (optional, [P][N]) receives the diagonal of the unnormalised A
pl_status launch_coherence(const PlaneTable& t, int N, const Geometry& g, const uint32_t* mask,
                           int prec, float2* coh, float* diag, hipStream_t s);
pl_status launch_phase_link(const float2* coh, int N, int64_t npix, int ref, int method,
                            float2* phasors, float* phase, float* lambda, uint8_t* flags,
                            unsigned long long* counters, hipStream_t s);
// adjoint of coherence + linking: per-pixel S = Abar + Abar^H (upper
// triangle, entry-major [N(N+1)/2][P]) from the recomputed coherence, then
// grad z_q = sum over the windows holding q as an SHP of S_p z_q
pl_status launch_link_vjp(const float2* coh, const float* diag, const uint8_t* flags,
                          const float* grad_phase, int N, int64_t npix, int ref, float2* S,
                          hipStream_t s);
pl_status launch_vjp_gather(const PlaneTable& t, int N, const Geometry& g, const uint32_t* mask,
                            const float2* S, float2* grad, hipStream_t s);
pl_status launch_compress(const PlaneTable& t, int N, int first_real, const Geometry& g,
                          const float2* phasors, float2* kappa, hipStream_t s);

}  // namespace plk
