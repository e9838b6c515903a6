/*
 * plink.h - C ABI of the MI355X (gfx950) sequential phase-linking library.
 *
 * Method: Staniewicz et al., "Near-Real-Time InSAR Phase Estimation for
 * Large-Scale Surface Displacement Monitoring" (arXiv 2511.12051).  Each call
 * below names the passage of the paper that defines what it computes.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Array arguments are DEVICE pointers into memory owned by the caller (for
 *    example PyTorch tensors); the library never frees or keeps them.  Host
 *    pointers are marked "host".
 *  - Complex numbers are pl_c64 = {float re; float im;} (complex64 layout).
 *  - Rasters are image-major and row-major: a stack is [N][R][C], an image
 *    (plane) is [R][C], so consecutive columns are consecutive in memory.
 *  - Every compute call enqueues its kernels on `stream` (a hipStream_t;
 *    NULL = the legacy default stream) and returns without waiting for them.
 *    Argument errors are detected before anything is enqueued; a launch
 *    failure is returned as PL_ERR_HIP.  pl_last_error() gives a message.
 *  - Window geometry (pl_window): the SHP search window of a pixel holds all
 *    pixels within half_x columns and half_y rows of it, i.e. a
 *    (2*half_x+1) x (2*half_y+1) box (supplement table of SHP window sizes);
 *    pixels outside the image are not part of it.  Phase linking runs on a
 *    decimated output grid of oR = R / stride_y rows and oC = C / stride_x
 *    columns whose pixel (oy, ox) sits at image pixel
 *    (oy*stride_y + stride_y/2, ox*stride_x + stride_x/2) (Sec. 4: linking
 *    at every 6th and 3rd pixel from the centre of each decimation window).
 *  - SHP masks are [oR][oC][nwords] uint32 with nwords = ceil(W/32),
 *    W = (2*half_x+1)*(2*half_y+1); bit b (word b/32, bit b%32) is window
 *    offset b in row-major order starting at (-half_y, -half_x).
 *  - Stacks hold at most PL_MAX_N images; compressed SLCs come first, in
 *    chronological order, then the real SLCs of the mini-stack (Sec. 2.2).
 *  - Optional `counters` arguments are device arrays of PL_NUM_COUNTERS
 *    uint64 (caller-owned, caller-zeroed) that the kernels add to.
 */
#ifndef PLINK_H
#define PLINK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PL_MAX_N 32
#define PL_MAX_WINDOW 1024 /* largest W = (2hx+1)(2hy+1) */

typedef void* pl_stream; /* hipStream_t */

typedef struct {
    float re;
    float im;
} pl_c64;

typedef enum {
    PL_OK = 0,
    PL_ERR_INVALID_ARG = 1, /* NULL pointer, bad enum value, non-positive size */
    PL_ERR_SHAPE = 2,       /* sizes inconsistent with each other or the window */
    PL_ERR_UNSUPPORTED = 3, /* outside what the kernels handle (e.g. N > PL_MAX_N) */
    PL_ERR_HIP = 4,         /* a HIP runtime call or kernel launch failed */
    PL_ERR_WORKSPACE = 5,   /* buffer too small */
    PL_ERR_STATE = 6        /* driver state or checkpoint does not match */
} pl_status;

typedef struct {
    int32_t half_x, half_y;     /* search half-window (columns, rows) */
    int32_t stride_x, stride_y; /* output decimation (columns, rows) */
} pl_window;

typedef enum {
    PL_PREC_FP32 = 0,      /* coherence accumulated with FP32 products */
    PL_PREC_SPLIT_BF16 = 1 /* products of hi+lo BF16 splits, FP32 accumulation */
} pl_precision;

typedef enum {
    PL_LINK_EMI = 0, /* EMI, EVD where the |C| inversion fails */
    PL_LINK_EVD = 1  /* EVD for every pixel */
} pl_link_method;

/* per-pixel flags written by phase linking */
enum { PL_FLAG_EMI = 0, PL_FLAG_EVD = 1, PL_FLAG_INVALID = 2 };

/* indices into the optional counters array */
enum {
    PL_CNT_GLRT_BAND = 0,     /* pair tests with |T - threshold| < 1e-9 */
    PL_CNT_GLRT_RECHECK = 1,  /* pair tests decided by the exact log form */
    PL_CNT_EVD = 2,           /* pixels that fell back to EVD */
    PL_CNT_INVALID = 3,       /* pixels flagged invalid */
    PL_CNT_NOT_CONVERGED = 4, /* eigenvector iterations that hit the cap */
    PL_CNT_SHIFT_RETRY = 5,   /* shifts rejected by the inertia check */
    PL_CNT_ITERS = 6,         /* total eigenvector iterations */
    PL_CNT_ITER_HIST = 8,     /* 16 entries: pixels by iteration count (entry
                                 15: 15 or more), invalid pixels excluded */
    PL_NUM_COUNTERS = 24
};

/* Host copy of a counters array (Sec. 3.2 expects the inverse power method to
 * need "typically under 10 iterations"; the histogram shows how many did). */
typedef struct {
    int64_t glrt_band, glrt_recheck, evd_fallbacks, invalid, not_converged, shift_retries,
        iterations;
    int64_t iter_hist[16];
} pl_report;

/* ---------------------------------------------------------------- library */
const char* pl_version(void);
const char* pl_status_string(pl_status s);
/* Message of the last failing call on this host thread ("" if none). */
const char* pl_last_error(void);
/* Output grid of an R x C image (host helper; no device work). */
pl_status pl_output_grid(int64_t R, int64_t C, pl_window w, int64_t* oR, int64_t* oC);
/* Number of uint32 words per SHP mask, or 0 for an invalid window. */
int32_t pl_mask_words(pl_window w);
/* Waits for `stream`, then copies a device counters array (PL_NUM_COUNTERS
 * uint64) into *out (host).  Errors of earlier kernels on the stream surface
 * here as PL_ERR_HIP. */
pl_status pl_sync_report(pl_stream stream, const uint64_t* counters, pl_report* out);

/* -------------------------------------------------- amplitude statistics
 * Per-pixel mean and population variance of |z| over the M images of `slc`
 * [M][R][C] (Sec. 3.1: mu_A and sigma_A of the amplitude dispersion; the
 * ancillary statistics stored with each compressed SLC).  Accumulated in
 * FP64.  mean, var: [R][C] float64. */
pl_status pl_amplitude_stats(const pl_c64* slc, int32_t M, int64_t R, int64_t C, double* mean,
                             double* var, pl_stream stream);

/* Pooled mean and variance of G groups of statistics (eq. merged-mean and
 * eq. merged-variance).  means, vars: [G][R][C] float64; weights: host [G],
 * positive.  mean_out, var_out: [R][C]; they may alias group 0. */
pl_status pl_merge_amplitude_stats(const double* means, const double* vars, const double* weights,
                                   int32_t G, int64_t R, int64_t C, double* mean_out,
                                   double* var_out, pl_stream stream);

/* ------------------------------------------------------- SHP selection
 * GLRT selection of statistically homogeneous pixels (Sec. 3.1: a GLRT on
 * amplitude means and variances).  With the Rayleigh scale
 * s = (mean^2 + var)/2 of each pixel and n = n_eff samples,
 * T = 2n [2 ln((s_p+s_q)/2) - ln s_p - ln s_q]; q is an SHP of p iff
 * T <= chi2_1^{-1}(1 - alpha).  A pixel is always an SHP of itself; a pixel
 * whose s is not finite and positive is an SHP of no other pixel and has only
 * itself.  The decision is taken in FP64; tests within 1e-9 of the threshold
 * are counted in counters[PL_CNT_GLRT_BAND].
 * mask: [oR][oC][nwords] uint32; count: [oR][oC] uint16 (SHPs incl. itself);
 * counters: optional. */
pl_status pl_shp_select(const double* mean, const double* var, int64_t R, int64_t C, double n_eff,
                        pl_window w, double alpha, uint32_t* mask, uint16_t* count,
                        uint64_t* counters, pl_stream stream);

/* --------------------------------------------------- sample coherence
 * Sample coherence over each output pixel's SHPs (eq. sample-coherence),
 * A_mn = sum_{q in Omega} z_m(q) conj(z_n(q)), normalised to unit diagonal:
 * C_mn = A_mn / sqrt(A_mm A_nn).  stack: [N][R][C]; mask as above;
 * coh: [oR*oC][N][N] full Hermitian matrices, row-major.  A pixel where some
 * image has zero power over its SHPs gets an all-NaN matrix.  prec selects
 * plain FP32 products or hi+lo BF16 split products on the matrix cores. */
pl_status pl_estimate_coherence(const pl_c64* stack, int32_t N, int64_t R, int64_t C, pl_window w,
                                const uint32_t* mask, pl_precision prec, pl_c64* coh,
                                pl_stream stream);

/* ------------------------------------------------------- phase linking
 * EMI phase linking (Sec. 3.2, eq. emi-eigenvalue-problem): the eigenvector
 * of the smallest eigenvalue of |C|^{-1} o C, found by shifted inverse
 * iteration starting from the shift 0.99; |C| is inverted in FP64 and when an
 * LDL^T pivot of |C| is <= 1e-6 (inversion fails) the pixel falls back to EVD,
 * the eigenvector of the largest eigenvalue of C.  The result is referenced to
 * image ref_idx (Sec. 2.1: multiplied by conj(zeta_r)) and returned as unit
 * phasors.  coh: [npix][N][N]; phasors: [N][npix] (phasors[ref_idx] = 1);
 * phase: [N][npix] or NULL, the same result as angles in (-pi, pi] (0 at
 * ref_idx and at invalid pixels); lambda: [npix] or NULL (eigenvalue of the vector: lambda_min of
 * |C|^{-1} o C for EMI, lambda_max of C for EVD); temp_coh: [npix] or NULL,
 * the temporal coherence of the result (Sec. 3.3, eq. temporal-coherence):
 * |sum_{i<k} exp(j(arg C_ik - (phi_i - phi_k)))| / (N(N-1)/2), with arg 0 = 0,
 * 1 for N = 1 and 0 at invalid pixels; flags: [npix] or NULL (PL_FLAG_*);
 * invalid pixels (non-finite C) get phasors 1.  For N > 16 C is read as the
 * Hermitian matrix of its upper triangle.  The iteration of a pixel stops when
 * its unit iterate changes by less than 2e-6 (or contracts fast enough for
 * the remaining error to be below that) and after at most 96 steps; a pixel
 * that reaches the cap keeps its last iterate and its normal flag, and is
 * counted in counters[PL_CNT_NOT_CONVERGED] (a few per million pixels on the
 * synthetic workloads).
 * counters: optional.  npix = 0 is a no-op (pointers may then be NULL). */
pl_status pl_phase_link(const pl_c64* coh, int32_t N, int64_t npix, int32_t ref_idx,
                        pl_link_method method, pl_c64* phasors, float* phase, float* lambda,
                        float* temp_coh, uint8_t* flags, uint64_t* counters, pl_stream stream);

/* ------------------------------------- fused coherence + phase linking
 * The sample coherence (eq. sample-coherence) of every output pixel linked
 * straight away (Sec. 3.2) without a full-size coherence array: the output
 * rows are processed in bands whose matrices, as packed upper triangles
 * (N(N+1)/2 entries per pixel), live only in `workspace`.  Inputs as for
 * pl_estimate_coherence; outputs as for pl_phase_link with npix = oR*oC
 * (phasors / phase [N][oR*oC], lambda / temp_coh / flags [oR*oC], each
 * optional except phasors).  The result equals pl_estimate_coherence followed
 * by pl_phase_link, except that every N reads C as the Hermitian matrix of its
 * upper triangle (for N <= 16 the two-step path reads full rows: the results
 * then differ by the rounding of C's lower triangle).
 * pl_phase_link_fused_workspace gives the bytes of one output row (the
 * minimum) and of all rows; a workspace of B bytes processes
 * B / min_bytes rows per band.  Errors: PL_ERR_WORKSPACE when ws_bytes <
 * min_bytes. */
pl_status pl_phase_link_fused_workspace(int32_t N, int64_t R, int64_t C, pl_window w, size_t* min_bytes,
                                        size_t* all_rows_bytes);
pl_status pl_phase_link_fused(const pl_c64* stack, int32_t N, int64_t R, int64_t C, pl_window w,
                              const uint32_t* mask, pl_precision prec, int32_t ref_idx,
                              pl_link_method method, pl_c64* phasors, float* phase, float* lambda,
                              float* temp_coh, uint8_t* flags, uint64_t* counters, void* workspace,
                              size_t ws_bytes, pl_stream stream);

/* ------------------------------------------- adjoint of coherence + link
 * Vector-Jacobian product of the linked phases phi_i = arg(v_i conj(v_ref))
 * with respect to the stack, through the sample coherence and the EMI / EVD
 * eigenvector (Sec. 2.1 eq. sample-coherence, Sec. 3.2
 * eq. emi-eigenvalue-problem), with the SHP mask and each pixel's EMI/EVD
 * choice held fixed (both are piecewise constant in the stack).  Per pixel,
 * with A = sum z z^H over the SHPs, C = D^-1/2 A D^-1/2, G = |C|,
 * H = G^-1 o C (EMI) or -C (EVD) and (v, lambda) its smallest eigenpair:
 *   dphi_i = Im(dv_i / v_i) - Im(dv_ref / v_ref),
 *   dv = -(H - lambda I)^+ dH v,  dH = -(G^-1 dG G^-1) o C + G^-1 o dC,
 *   dG = Re(conj(C) o dC) / |C|,  dA = sum (dz z^H + z dz^H).
 * The coherence and the eigenpair are recomputed here (prec must be the one
 * of the forward pass so that C is the same).
 * stack: [N][R][C]; mask: [oR][oC][nwords]; flags: [oR*oC] from
 * pl_phase_link (PL_FLAG_INVALID pixels contribute nothing); grad_phase:
 * [N][oR*oC] float, dL/dphi; grad_stack: [N][R][C] written (not accumulated)
 * with dL/dRe z + j dL/dIm z.  workspace: device memory of at least
 * pl_phase_link_vjp_workspace() bytes, owned by the caller, contents
 * irrelevant on entry.  Pixels whose value z is not finite get non-finite
 * gradients.  Errors: PL_ERR_WORKSPACE when ws_bytes is too small. */
pl_status pl_phase_link_vjp_workspace(int32_t N, int64_t R, int64_t C, pl_window w, size_t* bytes);
pl_status pl_phase_link_vjp(const pl_c64* stack, int32_t N, int64_t R, int64_t C, pl_window w,
                            const uint32_t* mask, const uint8_t* flags, int32_t ref_idx,
                            pl_precision prec, const float* grad_phase, pl_c64* grad_stack,
                            void* workspace, size_t ws_bytes, pl_stream stream);

/* The same vector-Jacobian product with every step in FP64: the sample
 * coherence accumulated in FP64 from the complex64 stack (each product of two
 * FP32 values is exact in FP64), |C| inverted and the eigenpair of
 * |C|^-1 o C (or -C) found by shifted inverse iteration in FP64, and the
 * pseudo-inverse solve, Gbar and the gather in FP64; grad_stack is rounded
 * to complex64 at the end.  Meant for derivatives that must match finite
 * differences of an FP64 evaluation (the FP32 call is limited by the FP32
 * eigen-solve).  flags hold the EMI/EVD choice fixed as above; an EMI pixel
 * whose |C| has an LDL^T pivot <= 1e-6 in FP64 contributes nothing.
 * workspace: at least pl_phase_link_vjp64_workspace() bytes
 * (N(N+1)/2 * oR*oC * 16).  Errors as pl_phase_link_vjp. */
pl_status pl_phase_link_vjp64_workspace(int32_t N, int64_t R, int64_t C, pl_window w, size_t* bytes);
pl_status pl_phase_link_vjp64(const pl_c64* stack, int32_t N, int64_t R, int64_t C, pl_window w,
                              const uint32_t* mask, const uint8_t* flags, int32_t ref_idx, const float* grad_phase,
                              pl_c64* grad_stack, void* workspace, size_t ws_bytes, pl_stream stream);

/* ------------------------------------------------------ compressed SLC
 * Compressed SLC of a mini-stack (Sec. 2.2): kappa = zeta^H z over the real
 * images first_real..N-1, i.e. kappa(p) = sum_i conj(zeta_i(b(p))) z_i(p),
 * where b(p) is the output pixel whose decimation block holds p
 * (b = (min(y/stride_y, oR-1), min(x/stride_x, oC-1))).
 * stack: [N][R][C]; phasors: [N][oR][oC]; kappa: [R][C]. */
pl_status pl_compress_ministack(const pl_c64* stack, int32_t N, int32_t first_real, int64_t R,
                                int64_t C, pl_window w, const pl_c64* phasors, pl_c64* kappa,
                                pl_stream stream);

/* The same as pl_phase_link_fused for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the bands go through a library-owned 128 MiB device
 * buffer, one per GPU, held until the process ends; the call allocates
 * nothing.  Every call on one GPU uses that GPU's buffer, so calls that
 * overlap on one GPU (other streams, other host threads) race: serialise
 * them.  Errors: PL_ERR_WORKSPACE when one output row of packed coherence
 * (oC * N(N+1)/2 * 8 bytes) exceeds the buffer. */
pl_status pl_phase_link_fused_noalloc(const pl_c64* stack, int32_t N, int64_t R, int64_t C, pl_window w,
                                      const uint32_t* mask, pl_precision prec, int32_t ref_idx,
                                      pl_link_method method, pl_c64* phasors, float* phase, float* lambda,
                                      float* temp_coh, uint8_t* flags, uint64_t* counters, pl_stream stream);

/* -------------------------------------- products of the linked phases */

/* Persistent scatterers and regridding to the output grid (Sec. 3.1: the
 * amplitude dispersion D_A = sigma_A / mu_A; Sec. 4: a threshold of 0.2;
 * supplement "Regridding PS and DS to 30 m resolution").  A pixel is a PS
 * iff mean > 0 and D_A <= da_threshold (D_A formed in FP64 from mean, var
 * [R][C] float64, e.g. pl_amplitude_stats or the merged statistics).  Each
 * output pixel takes the phasors ds_phasors [N][oR*oC] (its DS solution)
 * when its block (the full-resolution pixels mapped to it as in
 * pl_compress_ministack) holds no PS, else the single-reference phase
 * z_i conj(z_ref_idx) of the block's PS with the lowest D_A (the first in
 * row-major order on a tie) as unit phasors.  stack: [N][R][C];
 * out_phasors: [N][oR*oC], may equal ds_phasors; ps_source: [oR*oC] int64
 * flat index of the chosen PS or -1, or NULL; ps_mask: [R][C] uint8 (1 =
 * PS), or NULL. */
pl_status pl_ps_regrid(const pl_c64* stack, int32_t N, int64_t R, int64_t C, pl_window w, int32_t ref_idx,
                       const double* mean, const double* var, double da_threshold, const pl_c64* ds_phasors,
                       pl_c64* out_phasors, int64_t* ps_source, uint8_t* ps_mask, pl_stream stream);

/* Phase cosine similarity gamma_s (Sec. 3.3, eq. phase-cosine-sim) of linked
 * phasors [N][oR*oC] on the output grid: for every neighbour q of p inside
 * the disk of `radius` output pixels (1..15; p itself, pixels outside the grid
 * and pixels whose flag is PL_FLAG_INVALID excluded),
 * s = mean over the nearest-k network (pairs (a, b), 1 <= b - a <= k,
 * k = 1..3; Sec. 3.4) of cos((phi_a - phi_b)(p) - (phi_a - phi_b)(q)), and
 * gamma_s(p) is the median of these s (mean of the two middle values for an
 * even count); 0 for an invalid p or one without neighbours.  flags: [oR*oC]
 * or NULL; gamma_s: [oR*oC] float. */
pl_status pl_phase_similarity(const pl_c64* phasors, int32_t N, int64_t oR, int64_t oC, const uint8_t* flags,
                              int32_t radius, int32_t k, float* gamma_s, pl_stream stream);

/* Interferograms of the nearest-k network of N dates (Sec. 3.4: 3N - 6 for
 * k = 3), in the order the inversion reads them: by separation d = 1..k,
 * then by first date a (pairs (a, a + d)).  Host helper. */
pl_status pl_network_size(int32_t N, int32_t k, int32_t* n_ifg);

/* L1 network inversion (Sec. 3.5, eq. l1-min): for every pixel, x in
 * R^(N-1) (phases of dates 1..N-1 relative to date 0) minimising
 * ||A x - b||_1, A the incidence matrix of the network (row of pair (a, b):
 * +1 at date b, -1 at date a), by `iters` iterations of the ADMM of
 * Appendix A from z = u = 0 with parameter rho, the Cholesky factor of A^T A
 * shared by all pixels.  ifg: [n_ifg][P] float unwrapped interferogram
 * phases (order of pl_network_size); x: [N-1][P] float; residual_l1: [P]
 * float ||A x - b||_1 or NULL.  N = 2..32, k = 1..3; P = 0 is a no-op. */
pl_status pl_network_invert_l1(const float* ifg, int32_t N, int32_t k, int64_t P, double rho, int32_t iters,
                               float* x, float* residual_l1, pl_stream stream);

/* ----------------------------------------------- sequential estimator
 * The mini-stack reference scheme of Sec. 2.2 (Fig. 1, "proposed
 * approach"): mini-stack k is [kappa_{k-K} .. kappa_{k-1} | M new SLCs]
 * with K = min(k, K_max); it is referenced to the most recent compressed SLC
 * (to its first image for k = 0), so every output is referenced to the first
 * date; earlier mini-stacks are never re-estimated.  The amplitude
 * statistics of mini-stacks k-K..k are merged (eq. merged-mean/-variance)
 * with weights M decay^age (age 0 = the current mini-stack; Sec. 3.1: even
 * weights for decay = 1, an exponential decay that prioritises recent
 * observations below 1) and n_eff = the sum of the weights feeds the GLRT.
 * With reference = PL_SEQ_REF_LAST each compressed SLC is formed with the
 * phasors re-referenced to the last real SLC of its mini-stack, so mini-stack
 * k >= 1 is referenced to the last date of mini-stack k-1 (supplement,
 * "Compressed SLC strategy for separate batched processing"). */
enum { PL_SEQ_REF_COMPRESSED = 0, PL_SEQ_REF_LAST = 1 };
typedef struct pl_seq pl_seq;

typedef struct {
    int64_t R, C;       /* image size */
    int32_t M;          /* new SLCs per mini-stack (1..PL_MAX_N) */
    int32_t K_max;      /* compressed SLCs kept (M + K_max <= PL_MAX_N) */
    pl_window w;
    double alpha;       /* GLRT false-alarm rate */
    int32_t precision;  /* pl_precision */
    int32_t method;     /* pl_link_method */
    int32_t reference;  /* PL_SEQ_REF_* */
    double weight_decay; /* in (0, 1]; 1 = even weights */
} pl_seq_params;

/* Bytes of device state a driver with these parameters needs (host call):
 * the ring of K_max compressed SLCs, K_max + 1 per-mini-stack amplitude
 * statistics and the merged ones, and the intermediates of one mini-stack
 * (masks, counts, coherence, phasors, flags).  Errors as pl_seq_create. */
pl_status pl_seq_workspace_size(const pl_seq_params* params, size_t* bytes);
/* Creates a driver whose device state lives in the caller's buffer
 * (device memory, 256-byte aligned, at least pl_seq_workspace_size bytes).
 * The caller keeps ownership: the buffer must outlive the driver and is never
 * freed by it; the driver allocates no device memory.  PL_ERR_WORKSPACE if
 * the buffer is too small, PL_ERR_INVALID_ARG if it is NULL or misaligned. */
pl_status pl_seq_create_in(const pl_seq_params* params, void* dev_workspace, size_t bytes, pl_seq** out);
/* Creates a driver that allocates its device state (one block of
 * pl_seq_workspace_size bytes) on the current device and frees it in
 * pl_seq_destroy. */
pl_status pl_seq_create(const pl_seq_params* params, pl_seq** out);
pl_status pl_seq_destroy(pl_seq* s);
/* Number of mini-stacks pushed so far (host). */
pl_status pl_seq_count(const pl_seq* s, int64_t* count);
/* Processes the next mini-stack.  new_slcs: [M][R][C]; phasors_out:
 * [M][oR][oC] linked phasors of the new SLCs, referenced to the first date;
 * kappa_out: [R][C] or NULL (copy of the new compressed SLC); flags_out:
 * [oR*oC] or NULL; counters optional. */
pl_status pl_seq_push(pl_seq* s, const pl_c64* new_slcs, pl_c64* phasors_out, pl_c64* kappa_out,
                      uint8_t* flags_out, uint64_t* counters, pl_stream stream);
/* SHP masks ([oR][oC][nwords] uint32) of the most recent mini-stack, for
 * inspection (enqueued on `stream`).  PL_ERR_STATE before the first push. */
pl_status pl_seq_last_mask(const pl_seq* s, uint32_t* mask, pl_stream stream);
/* Size in bytes of a checkpoint (compressed SLCs, statistics, counters). */
pl_status pl_seq_state_size(const pl_seq* s, size_t* bytes);
/* Writes the checkpoint into host memory (synchronises `stream`). */
pl_status pl_seq_save(const pl_seq* s, void* host_buf, size_t bytes, pl_stream stream);
/* Restores a checkpoint written by a driver with the same parameters. */
pl_status pl_seq_load(pl_seq* s, const void* host_buf, size_t bytes, pl_stream stream);

/* ------------------------------------------- batched, graph-replayed runs
 * Several independent mini-stacks, for instance the next mini-stack of many
 * bursts, each with its own number of compressed SLCs and hence its own N,
 * go through the whole path of Sec. 2.2 / 3.1 / 3.2 (amplitude statistics,
 * GLRT SHPs, sample coherence, EMI/EVD linking, compressed SLC) with one
 * persistent launch per stage and kernel variant: each launch strides over
 * the workgroups of all the items that share its variant.  pl_batch_plan
 * checks the items, allocates the intermediates (SHP masks, coherence,
 * statistics when not supplied) on the current device and, with autotune,
 * times a few strip widths / rows per workgroup of the coherence kernel and
 * grid sizes of the linking kernel on the items' current contents (so fill
 * the inputs first) and keeps the fastest.  The first pl_batch_run on a stream
 * captures the launches into a HIP graph; later runs replay it, so every
 * pointer of the plan must stay valid and inputs are refilled in place.
 * Levels chain mini-stacks: the sequential scheme of Sec. 2.2 over several
 * bursts is one plan whose level k holds mini-stack k of every burst, its
 * planes pointing at the kappa outputs of levels < k (statistics merged
 * beforehand, e.g. with pl_merge_amplitude_stats, since they do not depend on
 * the linking).  Results are identical to the single-call entry points. */
typedef struct {
    const pl_c64* stack;  /* [N][R][C]: first_real compressed SLCs, then real images */
    int64_t R, C;
    int32_t N;            /* 1..PL_MAX_N */
    int32_t first_real;   /* 0..N-1 */
    int32_t ref_idx;      /* reference image, 0..N-1 */
    const double* mean;   /* [R][C] amplitude mean and variance for the GLRT, or */
    const double* var;    /* NULL: computed from the real images */
    double n_eff;         /* GLRT sample count; <= 0: N - first_real */
    pl_c64* phasors;      /* [N][oR][oC] out */
    uint8_t* flags;       /* [oR*oC] out, or NULL */
    pl_c64* kappa;        /* [R][C] compressed SLC out, or NULL */
    const pl_c64* const* planes;  /* host array of N device pointers to the
                                     [R][C] images (used instead of stack), or NULL */
    int32_t level;        /* items run level by level in increasing order; a
                             level may read the kappa of lower levels */
} pl_batch_item;

typedef struct pl_batch pl_batch;

pl_status pl_batch_plan(const pl_batch_item* items, int32_t n_items, pl_window w, double alpha,
                        pl_precision prec, pl_link_method method, int32_t autotune,
                        pl_stream stream, pl_batch** out);
pl_status pl_batch_run(pl_batch* b, pl_stream stream);
pl_status pl_batch_destroy(pl_batch* b);
/* Text summary of the plan: launches, kernel variants, tiles, grid sizes and
 * (after a run) whether a graph is held.  Writes at most len bytes. */
pl_status pl_batch_describe(const pl_batch* b, char* buf, size_t len);
/* Chooses how pl_batch_run executes the plan (host call; synchronises the
 * plan's stream and drops a captured graph).  on != 0: the whole run as ONE
 * persistent launch (the default whenever the plan supports it): every
 * (item, stage) pair is a segment of work units in one device-wide queue,
 * in dependency order, and a workgroup starts a segment only after the
 * segments it depends on are complete (the item's previous stage; for
 * coherence also the compression of each item whose compressed SLC it reads,
 * Sec. 2.2, Fig. 1).  on == 0: one persistent launch per stage and kernel
 * variant, as above.  Both forms give bit-identical results.
 * PL_ERR_UNSUPPORTED when the plan cannot run as one launch (pl_batch_describe
 * gives the reason: a tile that does not fit one 512-thread workgroup). */
pl_status pl_batch_set_single_launch(pl_batch* b, int32_t on);
/* Synchronises `stream` and the plan's stream; PL_ERR_STATE if a
 * single-launch run since the previous check waited past its bound (about
 * 0.25 s per wait; the run then completed without its ordering guarantee,
 * so its outputs are not to be used). */
pl_status pl_batch_check(pl_batch* b, pl_stream stream);
/* Sets the bound of every wait of the single launch, in sleep rounds of about
 * 0.2 us (default 2^20); drops a captured graph.  A bound of 0 makes every
 * wait give up at once: the run still ends and pl_batch_check reports it,
 * which is how the failure path is tested without stalling a GPU. */
pl_status pl_batch_set_wait_limit(pl_batch* b, uint32_t spins);

#ifdef __cplusplus
}
#endif

#endif /* PLINK_H */
