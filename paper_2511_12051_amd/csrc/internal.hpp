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

// ---- per-launch arguments of the stage kernels (one per item in batched
// launches, see batch_device.hpp)
struct StatsArgs {
    PlaneTable t;
    int first, M;
    int64_t n;  // pixel pairs (16-byte variant) or pixels
    double* mean;
    double* var;
};

struct GlrtArgs {
    const double* mean;
    const double* var;
    Geometry g;
    int TX, TY, tw, th;
    double n, thr, rlo, rhi;
    uint32_t* mask;
    uint16_t* count;
    unsigned long long* counters;
    int64_t gx;  // tiles per tile row
};

struct CohArgs {
    PlaneTable t;
    int N;
    Geometry g;
    const uint32_t* mask;
    float2* coh;      // [P][N][N], or [P][N(N+1)/2] upper triangles when packed
    float* diag;      // optional [P][N] diagonal of A (SHP-summed |z|^2), or null
    int packed;       // write each matrix as its packed upper triangle
    int64_t oy_lo, oy_hi;  // output rows of this launch; pixel p of coh is
                           // (oy_lo + p / oC, p % oC)
    int TXo;          // output columns per strip
    int rows_per_wg;  // output rows per workgroup
    int tile_w;       // staged input columns (even)
    int pitch;        // records (pixel pairs) per staged row = tile_w / 2
    int plane;        // records per image plane (wy * pitch, padded)
    int wave_words;   // 32-bit words of LDS per wavefront
    int n_pairs;      // pairs per window = (2 hy + 1)(hx + 1)
    float inv_ppr;    // 1 / (hx + 1), for exact small divisions
    int vec_rows;     // every image row starts 16-byte aligned (pairs load as 16 bytes)
    int64_t n_strips; // strips of TXo output columns (batched launches)
};

struct LinkArgs {
    const float2* coh;  // [npix][N][N], or packed upper triangles [npix][N(N+1)/2]
    int N;
    int64_t npix;
    int ref;
    int method;
    float2* ph;         // [N][ostride] (pixel p of image i at ph[i * ostride + p])
    float* phase;       // optional, same layout: angles in (-pi, pi], 0 at the reference
    float* lam;         // optional [npix]
    uint8_t* flags;     // optional [npix]
    unsigned long long* counters;
    float* tcoh;        // optional [npix] temporal coherence of the linked phases
    int packed;         // coh layout
    int64_t ostride;    // image stride of ph / phase (>= npix)
};

struct CompressArgs {
    PlaneTable t;
    int N, first_real;
    Geometry g;
    const float2* ph;
    float2* kappa;
    int64_t gx;  // blocks per image row
    int rot;     // >= 0: kappa multiplied by phasor rot of its block (re-reference)
};

template <typename Args>
struct BatchRange;

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
// output rows [oy_lo, oy_hi) only, optionally as packed upper triangles
pl_status launch_coherence_rows(const PlaneTable& t, int N, const Geometry& g, const uint32_t* mask,
                                int prec, float2* coh, int packed, int64_t oy_lo, int64_t oy_hi,
                                hipStream_t s);
pl_status launch_coherence_args(CohArgs& a, int prec, hipStream_t s);  // a: t, N, g, mask, coh, diag,
                                                                       // packed, oy_lo, oy_hi set
pl_status launch_phase_link(const LinkArgs& a, hipStream_t s);
LinkArgs link_args(const float2* coh, int N, int64_t npix, int ref, int method, float2* phasors,
                   float* phase, float* lambda, uint8_t* flags, unsigned long long* counters);
// adjoint of coherence + linking: per-pixel S = Abar + Abar^H (upper
// triangle, entry-major [N(N+1)/2][P]) from the recomputed coherence, then
// grad z_q = sum over the windows holding q as an SHP of S_p z_q
pl_status launch_link_vjp(const float2* coh, const float* diag, const uint8_t* flags,
                          const float* grad_phase, int N, int64_t npix, int ref, float2* S,
                          hipStream_t s);
pl_status launch_vjp_gather(const PlaneTable& t, int N, const Geometry& g, const uint32_t* mask,
                            const float2* S, float2* grad, hipStream_t s);
pl_status launch_compress(const PlaneTable& t, int N, int first_real, const Geometry& g,
                          const float2* phasors, float2* kappa, hipStream_t s, int rot = -1);

// ---- argument set-up and batched (persistent, multi-item) launches
bool stats_args(const PlaneTable& t, int first, int M, int64_t npix, double* mean, double* var,
                StatsArgs* a, int64_t* blocks);  // returns whether the 16-byte variant applies
bool glrt_args(const double* mean, const double* var, const Geometry& g, double n_eff, double alpha,
               uint32_t* mask, uint16_t* count, unsigned long long* counters, GlrtArgs* a,
               int64_t* blocks, size_t* lds);  // false when the tile does not fit in LDS
// tile set-up of one coherence launch: txo_max caps the strip width, rows (> 0)
// overrides the output rows per workgroup; returns the dynamic LDS bytes
// (0: does not fit) and the number of workgroups
size_t coherence_args(CohArgs* a, int nt, bool split, int txo_max, int rows, int64_t* blocks);
CompressArgs compress_args(const PlaneTable& t, int N, int first_real, const Geometry& g,
                           const float2* phasors, float2* kappa, int64_t* blocks);
int64_t link_blocks(int N, int64_t npix);  // workgroups of one linking launch

// kernel entry points of the batched launches (occupancy queries, LDS limits)
const void* amp_stats_batch_fn(bool vec);
const void* glrt_batch_fn();
const void* coherence_batch_fn(int nt, bool split);
int coherence_threads(int nt);  // workgroup size of the coherence kernels
int coherence_strip(int nt);    // default output columns per strip
const void* phase_link_batch_fn(int N_class);
const void* compress_batch_fn();
pl_status allow_dynamic_lds(const void* fn, size_t lds);

pl_status launch_amp_stats_batch(const BatchRange<StatsArgs>& r, bool vec, int64_t grid, hipStream_t s);
pl_status launch_shp_select_batch(const BatchRange<GlrtArgs>& r, int threads, size_t lds, int64_t grid,
                                  hipStream_t s);
pl_status launch_coherence_batch(const BatchRange<CohArgs>& r, int nt, bool split, size_t lds, int64_t grid,
                                 hipStream_t s);
pl_status launch_phase_link_batch(const BatchRange<LinkArgs>& r, int N_class, int64_t grid, hipStream_t s);
pl_status launch_compress_batch(const BatchRange<CompressArgs>& r, int64_t grid, hipStream_t s);

// ---- the whole batched run as one persistent launch: a queue of work units
// in dependency order (stage segments of every item), each segment's
// completions counted in device memory, every wait bounded
enum MegaStage {
    MS_STATS_VEC = 0, MS_STATS_SCALAR, MS_GLRT, MS_COH16, MS_COH32,
    MS_LINK = 8,                  // + linking class (N + 3) / 4, 1..8
    MS_COMPRESS = MS_LINK + 9,
};
constexpr int kMegaMaxDeps = 8;
struct MegaSeg {
    int stage;        // MegaStage
    int arg;          // index into the stage's argument table
    int64_t blocks;   // blocks of the stage's own kernel for this item
    int per_unit;     // of those, per work unit
    int64_t units;
    int ndep;
    int dep[kMegaMaxDeps];  // earlier segments that must be complete first
};
struct MegaPlan {
    const MegaSeg* seg;
    const int64_t* seg_start;  // nseg + 1 prefix sums of units
    int nseg;
    int64_t total;             // work units per run
    const StatsArgs* stats;
    const GlrtArgs* glrt;
    const CohArgs* coh;
    const LinkArgs* link;
    const CompressArgs* comp;
    unsigned long long* queue;  // units handed out, over all runs
    unsigned long long* done;   // [nseg] completed units, over all runs
    unsigned int* run;          // completed runs
    unsigned int* finished;     // workgroups finished, over all runs
    unsigned int* error;        // set when a wait exceeded spin_limit
    unsigned int spin_limit;
};
int mega_threads();
const void* mega_fn(bool split);
size_t mega_link_lds(int N_class);  // LDS of one work unit of a linking class
pl_status launch_mega(const MegaPlan& p, bool split, size_t lds, int64_t grid, hipStream_t s);

}  // namespace plk
