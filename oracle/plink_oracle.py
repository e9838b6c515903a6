"""Plain FP64 CPU oracle for the sequential phase-linking hot path.

TEST INFRASTRUCTURE ONLY.  This module is the checker that the GPU library is
measured against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product path
(``paper_2511_12051_amd``) never does, and shares no code with it.

Everything is computed in float64 / complex128 with NumPy (and SciPy for the
chi-square quantile and nothing else).  Loops run over window offsets and
matrix indices exactly as the definitions read; the only vectorisation is over
independent output pixels.

Source: Staniewicz et al., "Near-Real-Time InSAR Phase Estimation for
Large-Scale Surface Displacement Monitoring" (arXiv 2511.12051).  Citations
name the section / equation / figure / table of that paper.

Readings taken where the paper is silent (each one is listed in the design doc):

* R1 output grid: oR = R // s_y, oC = C // s_x; output pixel (oy, ox) sits at
  (oy*s_y + s_y//2, ox*s_x + s_x//2) ("every 6th and 3rd pixel", Sec. 4
  processing configuration; "center of the decimation window", supplement on
  PS/DS regridding).  Window = all pixels within half_x columns and half_y rows
  of the centre (supplement table of SHP window sizes: full = 2h+1); pixels
  outside the image are not part of the window.
* R2 GLRT form (Sec. 3.1 cites a GLRT that needs only amplitude means and
  variances, with no formula): Rayleigh amplitude model implied by the CCG
  model (Sec. 2.1).  Scale s = (mu^2 + sigma^2)/2 (the Rayleigh ML scale,
  sum|z|^2 / 2n), T = 2n[2 ln((s_p+s_q)/2) - ln s_p - ln s_q], SHP iff
  T <= chi2_1^{-1}(1 - alpha).  sigma^2 is the population variance, which makes
  the merged-variance equation exact.
* R3 coherence normalisation: the sample covariance (eq. sample-coherence) is
  normalised to unit diagonal, C = D^{-1/2} A D^{-1/2}, because Sec. 2.1
  assumes unit power and uses |Sigma| as the coherence magnitude.  The 1/L
  factor cancels.
* R4 conjugation: A_mn = sum z_m conj(z_n) (z z^H, the definition of Sigma in
  Sec. 2.1), so the linked phase of image i estimates phi_i - phi_r.
* R5 EMI/EVD fallback (Sec. 3.2 "inversion ... fails due to numerical
  issues"): EVD iff some LDL^T pivot of |C| is <= TAU_PIVOT or non-finite.
* R6 EMI/EVD vectors: the eigenvector of the smallest eigenvalue of
  |C|^{-1} o C (eq. emi-eigenvalue-problem), resp. of the largest eigenvalue of
  C (EVD), from a full Hermitian eigendecomposition.
* R7 compressed SLC at full resolution: each pixel uses the linked phases of
  its decimation block (nearest-block upsampling), kappa = zeta^H z over the
  real SLCs of the mini-stack (Sec. 2.2; a sum, not a mean).
* R8 sequential statistics: the amplitude statistics merged for mini-stack k
  are those of mini-stacks k-K..k (the ones behind the retained compressed
  SLCs plus the current one), each weighted by its number of images
  (eq. merged-mean / merged-variance, "evenly weight the previous n images").
* R18 exponential weights: the group of age a is weighted by M decay^a and
  the GLRT sample count is the sum of the weights (decay = 1: reading R8).
"""
from __future__ import annotations

import numpy as np
from scipy import stats as _scipy_stats

#: LDL^T pivot of |C| at or below which the |C| inversion is deemed to fail
#: (reading R5; |C| has unit diagonal so the pivots are on a scale of 1).
TAU_PIVOT = 1e-6

#: GLRT statistics within this distance of the threshold are "band" cases:
#: counted and reported, excluded from bit-exact mask comparison.
GLRT_BAND = 1e-9

#: flags returned by :func:`phase_link`
FLAG_EMI, FLAG_EVD, FLAG_INVALID = 0, 1, 2


# --------------------------------------------------------------------------
# geometry (reading R1)
# --------------------------------------------------------------------------
def output_grid(R: int, C: int, window) -> tuple[int, int]:
    """Output grid size (oR, oC) for an R x C image; window = (hx, hy, sx, sy)."""
    hx, hy, sx, sy = window
    return R // sy, C // sx


def output_centres(R: int, C: int, window):
    """Row and column index of every output pixel centre (reading R1)."""
    hx, hy, sx, sy = window
    oR, oC = output_grid(R, C, window)
    cy = np.arange(oR) * sy + sy // 2
    cx = np.arange(oC) * sx + sx // 2
    return cy, cx


def window_offsets(window):
    """Window offsets (dy, dx), row-major from (-hy, -hx); bit b of a SHP mask
    is offset number b of this list (word b // 32, bit b % 32)."""
    hx, hy = window[0], window[1]
    return [(dy, dx) for dy in range(-hy, hy + 1) for dx in range(-hx, hx + 1)]


def mask_words(window) -> int:
    hx, hy = window[0], window[1]
    return ((2 * hx + 1) * (2 * hy + 1) + 31) // 32


# --------------------------------------------------------------------------
# amplitude statistics (Sec. 3.1: D_A definition; eq. merged-mean/-variance)
# --------------------------------------------------------------------------
def amplitude_stats(slc):
    """Per-pixel mean and population variance of |z| over the images of
    ``slc`` [M, R, C] (the mu_A, sigma_A^2 of the amplitude dispersion)."""
    a = np.abs(np.asarray(slc).astype(np.complex128))
    mean = a.mean(axis=0)
    var = a.var(axis=0)  # ddof = 0: population variance (reading R2)
    return mean, var


def merge_amplitude_stats(means, variances, weights):
    """Pooled mean and variance of groups (eq. merged-mean, eq. merged-variance).

    means, variances: sequences of [R, C] arrays; weights: one weight per group.
    """
    w = np.asarray(weights, dtype=np.float64)
    wsum = w.sum()
    mu = sum(wi * np.asarray(m, dtype=np.float64) for wi, m in zip(w, means)) / wsum
    second = sum(wi * (np.asarray(v, dtype=np.float64) + np.asarray(m, dtype=np.float64) ** 2)
                 for wi, m, v in zip(w, means, variances)) / wsum
    return mu, second - mu ** 2


# --------------------------------------------------------------------------
# GLRT SHP selection (Sec. 3.1; reading R2)
# --------------------------------------------------------------------------
def glrt_threshold(alpha: float) -> float:
    """Chi-square (1 degree of freedom) quantile at 1 - alpha."""
    return float(_scipy_stats.chi2.isf(alpha, 1))


def rayleigh_scale(mean, var):
    """Rayleigh ML scale (mu^2 + sigma^2) / 2 = sum |z|^2 / (2n)."""
    return (np.asarray(mean, dtype=np.float64) ** 2 + np.asarray(var, dtype=np.float64)) / 2.0


def glrt_statistic(s_p, s_q, n):
    """GLRT for 'p and q share one Rayleigh scale' with n samples each."""
    s_p = np.asarray(s_p, dtype=np.float64)
    s_q = np.asarray(s_q, dtype=np.float64)
    return 2.0 * n * (2.0 * np.log((s_p + s_q) / 2.0) - np.log(s_p) - np.log(s_q))


def shp_select(mean, var, n, window, alpha, return_stat=False):
    """SHP masks of every output pixel.

    Returns (mask uint32 [oR, oC, nwords], count uint16 [oR, oC], band_count)
    and, with ``return_stat``, the statistic T [oR, oC, W] (NaN where the pair
    is not tested) so that tests can locate band cases.
    """
    R, C = np.shape(mean)
    oR, oC = output_grid(R, C, window)
    cy, cx = output_centres(R, C, window)
    offs = window_offsets(window)
    W = len(offs)
    nw = mask_words(window)
    thr = glrt_threshold(alpha)
    s = rayleigh_scale(mean, var)
    s_ok = np.isfinite(s) & (s > 0)

    CY, CX = np.meshgrid(cy, cx, indexing="ij")
    sp = s[CY, CX]
    sp_ok = s_ok[CY, CX]
    bits = np.zeros((oR, oC, W), dtype=bool)
    stat = np.full((oR, oC, W), np.nan)
    band = 0
    for b, (dy, dx) in enumerate(offs):
        qy, qx = CY + dy, CX + dx
        inside = (qy >= 0) & (qy < R) & (qx >= 0) & (qx < C)
        qyc, qxc = np.clip(qy, 0, R - 1), np.clip(qx, 0, C - 1)
        sq = s[qyc, qxc]
        tested = inside & sp_ok & s_ok[qyc, qxc]
        with np.errstate(all="ignore"):
            t = glrt_statistic(sp, sq, n)
        bits[..., b] = tested & (t <= thr)
        stat[..., b] = np.where(tested, t, np.nan)
        band += int(np.count_nonzero(tested & (np.abs(t - thr) < GLRT_BAND)))
        if dy == 0 and dx == 0:
            bits[..., b] = True  # the pixel itself always belongs to its own Omega
    mask = np.zeros((oR, oC, nw), dtype=np.uint32)
    for b in range(W):
        mask[..., b // 32] |= bits[..., b].astype(np.uint32) << np.uint32(b % 32)
    count = bits.sum(axis=-1).astype(np.uint16)
    if return_stat:
        return mask, count, band, stat
    return mask, count, band


def mask_bits(mask, window):
    """Unpack a [.., nwords] uint32 mask into booleans [.., W]."""
    W = (2 * window[0] + 1) * (2 * window[1] + 1)
    m = np.asarray(mask, dtype=np.uint32)
    out = np.zeros(m.shape[:-1] + (W,), dtype=bool)
    for b in range(W):
        out[..., b] = (m[..., b // 32] >> np.uint32(b % 32)) & 1
    return out


# --------------------------------------------------------------------------
# sample coherence (eq. sample-coherence; readings R3, R4)
# --------------------------------------------------------------------------
def coherence(stack, mask, window, pixels=None):
    """Normalised sample coherence over each output pixel's SHPs.

    stack [N, R, C]; mask [oR, oC, nwords].  ``pixels`` optionally restricts
    the result to a list of (oy, ox) output pixels.  Returns (C, valid) with C
    complex128 [P, N, N] (P = oR*oC row-major, or len(pixels)) and a boolean
    valid flag (False when some image has zero power over Omega).
    """
    z = np.asarray(stack).astype(np.complex128)
    N, R, C = z.shape
    cy, cx = output_centres(R, C, window)
    oR, oC = len(cy), len(cx)
    if pixels is None:
        oy, ox = np.meshgrid(np.arange(oR), np.arange(oC), indexing="ij")
        oy, ox = oy.ravel(), ox.ravel()
    else:
        pixels = np.asarray(pixels).reshape(-1, 2)
        oy, ox = pixels[:, 0], pixels[:, 1]
    bits = mask_bits(np.asarray(mask)[oy, ox], window)  # [P, W]
    P = len(oy)
    A = np.zeros((P, N, N), dtype=np.complex128)
    for b, (dy, dx) in enumerate(window_offsets(window)):
        qy, qx = cy[oy] + dy, cx[ox] + dx
        use = bits[:, b] & (qy >= 0) & (qy < R) & (qx >= 0) & (qx < C)
        if not use.any():
            continue
        zq = z[:, np.clip(qy, 0, R - 1), np.clip(qx, 0, C - 1)].T  # [P, N]
        zq = np.where(use[:, None], zq, 0)
        A += zq[:, :, None] * np.conj(zq[:, None, :])  # z z^H
    d = np.real(np.einsum("pii->pi", A))
    valid = np.all(np.isfinite(A.reshape(P, -1)), axis=1) & np.all(d > 0, axis=1)
    with np.errstate(all="ignore"):
        Cn = A / np.sqrt(d[:, :, None] * d[:, None, :])
    Cn[~valid] = np.nan
    return Cn, valid


# --------------------------------------------------------------------------
# EMI / EVD phase linking (Sec. 2.1 reference; Sec. 3.2; readings R5, R6)
# --------------------------------------------------------------------------
def ldl_pivots(G):
    """Pivots d_k of the unpivoted LDL^T factorisation of each real symmetric
    matrix in G [P, N, N] (d_k = squared Cholesky diagonal)."""
    A = np.array(G, dtype=np.float64, copy=True)
    P, N, _ = A.shape
    d = np.empty((P, N))
    with np.errstate(all="ignore"):
        for k in range(N):
            d[:, k] = A[:, k, k]
            l = A[:, k + 1:, k] / d[:, k, None]
            A[:, k + 1:, k + 1:] -= l[:, :, None] * l[:, None, :] * d[:, k, None, None]
            A[:, k + 1:, k] = l
    return d


def phase_link(Cmat, ref=0, method="emi", valid=None, tau=TAU_PIVOT):
    """Linked phasors of each coherence matrix.

    Cmat complex [P, N, N].  Returns a dict with
      phasor  complex128 [N, P]  unit modulus, phasor[ref] = 1
      phase   float64 [N, P]     angle in (-pi, pi]
      lam     float64 [P]        eigenvalue of the chosen vector
      flag    uint8 [P]          0 EMI, 1 EVD, 2 invalid
      min_pivot float64 [P]      smallest LDL^T pivot of |C| (EMI decision)
      cond    float64 [P]        ||B||_2 / eigen-gap of the matrix B solved
    """
    Cm = np.asarray(Cmat, dtype=np.complex128)
    P, N, _ = Cm.shape
    if valid is None:
        valid = np.all(np.isfinite(Cm.reshape(P, -1)), axis=1)
    valid = np.asarray(valid, dtype=bool).copy()
    Csafe = np.where(valid[:, None, None], Cm, np.eye(N))
    G = np.abs(Csafe)
    piv = ldl_pivots(G)
    min_piv = np.where(np.all(np.isfinite(piv), axis=1), piv.min(axis=1), -np.inf)
    emi_ok = min_piv > tau
    use_evd = np.ones(P, dtype=bool) if method == "evd" else ~emi_ok

    v = np.zeros((P, N), dtype=np.complex128)
    lam = np.zeros(P)
    cond = np.full(P, np.inf)
    e = valid & ~use_evd
    if e.any():
        H = np.linalg.inv(G[e]) * Csafe[e]
        H = 0.5 * (H + np.conj(np.swapaxes(H, 1, 2)))  # exact Hermitian part
        w, V = np.linalg.eigh(H)
        v[e] = V[:, :, 0]
        lam[e] = w[:, 0]
        if N > 1:
            cond[e] = np.abs(w).max(axis=1) / (w[:, 1] - w[:, 0])
    f = valid & use_evd
    if f.any():
        w, V = np.linalg.eigh(Csafe[f])
        v[f] = V[:, :, -1]
        lam[f] = w[:, -1]
        if N > 1:
            cond[f] = np.abs(w).max(axis=1) / (w[:, -1] - w[:, -2])
    vr = v[:, ref]
    valid &= np.abs(vr) > 0
    # multiplying by conj(zeta_r) sets phi_r = 0 (Sec. 2.1); the positive factor
    # 1/|v_r| does not change any angle
    zeta = v * np.conj(vr)[:, None]
    phase = np.angle(zeta)  # angle(0) = 0
    phase[:, ref] = 0.0     # exactly, not up to the rounding of |v_r|^2
    phase[~valid] = 0.0
    flag = np.where(use_evd, FLAG_EVD, FLAG_EMI).astype(np.uint8)
    flag[~valid] = FLAG_INVALID
    return {
        "phasor": np.exp(1j * phase).T.copy(),
        "phase": phase.T.copy(),
        "lam": lam,
        "flag": flag,
        "min_pivot": min_piv,
        "cond": cond,
    }


def phase_sensitivity(Cmat, ref=0, method="emi", n_probe=4, eps=1e-7, seed=0):
    """Statistical estimate of how far the linked phases move per unit change
    of the entries of C (test infrastructure, not part of the method).

    Each probe adds a random Hermitian perturbation with |E_mn| = eps off the
    diagonal (the diagonal stays 1) and re-links in FP64; the estimate is the
    largest wrapped phase change over probes and images divided by eps
    (small-sample statistical condition estimation).  Pixels whose EMI/EVD
    decision flips under a probe, or that are invalid, get inf.
    """
    Cm = np.asarray(Cmat, dtype=np.complex128)
    P, N, _ = Cm.shape
    base = phase_link(Cm, ref=ref, method=method)
    rng = np.random.default_rng(seed)
    sens = np.zeros(P)
    iu = np.triu_indices(N, 1)
    for _ in range(n_probe):
        E = np.zeros((P, N, N), dtype=np.complex128)
        th = rng.uniform(-np.pi, np.pi, (P, len(iu[0])))
        E[:, iu[0], iu[1]] = eps * np.exp(1j * th)
        E = E + np.conj(np.swapaxes(E, 1, 2))
        out = phase_link(Cm + E, ref=ref, method=method)
        d = np.abs(wrap(out["phase"] - base["phase"])).max(axis=0) / eps
        d[out["flag"] != base["flag"]] = np.inf
        sens = np.maximum(sens, d)
    sens[base["flag"] == FLAG_INVALID] = np.inf
    return sens


# --------------------------------------------------------------------------
# adjoint of coherence + phase linking (test oracle for the GPU adjoint)
# --------------------------------------------------------------------------
def link_phases_fixed(stack, mask, window, ref, flags, pixels=None):
    """Linked phases [N, P] with the SHP mask and the EMI/EVD choice held
    fixed (flags from an earlier phase_link) - the function the adjoint
    differentiates."""
    Cm, valid = coherence(stack, mask, window, pixels=pixels)
    emi = np.asarray(flags) == FLAG_EMI
    out = np.zeros((Cm.shape[1], Cm.shape[0]))
    if emi.any():
        out[:, emi] = phase_link(Cm[emi], ref=ref, method="emi", tau=-np.inf)["phase"]
    evd = np.asarray(flags) == FLAG_EVD
    if evd.any():
        out[:, evd] = phase_link(Cm[evd], ref=ref, method="evd")["phase"]
    return out


def phase_link_vjp(stack, mask, window, ref, grad_phase, flags):
    """Vector-Jacobian product of the linked phases with respect to the stack.

    grad_phase [N, P] is dL/dphi for every output pixel; returns dL/dz as a
    complex128 [N, R, C] array in the convention dL/dRe + j dL/dIm.  The SHP
    mask and the EMI/EVD choice (flags) are held fixed, invalid pixels
    contribute nothing.  Per pixel, with A = sum z z^H over the SHPs,
    C = D^-1/2 A D^-1/2, G = |C|, H = G^-1 o C (EMI) or H = -C (EVD) and v
    the eigenvector of the smallest eigenvalue lambda of H:
      phi_i = arg(v_i conj(v_r))       -> dL = Re(u^H dv)
      dv = -(H - lambda I)^+ dH v      -> Hbar = -y v^H, y = (H - lambda I)^+ u
      dH = -(G^-1 dG G^-1) o C + G^-1 o dC, dG = Re(conj(C) dC)/|C|
      C = A / sqrt(A_mm A_nn),  A = sum z z^H  -> grad z_q = (Abar + Abar^H) z_q.
    """
    z = np.asarray(stack).astype(np.complex128)
    N, R, Cc = z.shape
    cy, cx = output_centres(R, Cc, window)
    oR, oC = len(cy), len(cx)
    P = oR * oC
    offs = window_offsets(window)
    bits = mask_bits(np.asarray(mask).reshape(P, -1), window)
    oy, ox = np.meshgrid(np.arange(oR), np.arange(oC), indexing="ij")
    oy, ox = oy.ravel(), ox.ravel()
    A = np.zeros((P, N, N), dtype=np.complex128)
    for b, (dy, dx) in enumerate(offs):
        qy, qx = cy[oy] + dy, cx[ox] + dx
        use = bits[:, b] & (qy >= 0) & (qy < R) & (qx >= 0) & (qx < Cc)
        zq = np.where(use[:, None], z[:, np.clip(qy, 0, R - 1), np.clip(qx, 0, Cc - 1)].T, 0)
        A += zq[:, :, None] * np.conj(zq[:, None, :])
    d = np.real(np.einsum("pii->pi", A))
    flags = np.asarray(flags)
    grad = np.zeros_like(z)
    g = np.asarray(grad_phase, dtype=np.float64).reshape(N, P)
    S = np.zeros((P, N, N), dtype=np.complex128)
    for p in range(P):
        if flags[p] == FLAG_INVALID or not np.all(d[p] > 0):
            continue
        s = np.sqrt(np.outer(d[p], d[p]))
        Cp = A[p] / s
        if flags[p] == FLAG_EMI:
            G = np.abs(Cp)
            Gi = np.linalg.inv(G)
            H = Gi * Cp
        else:
            H = -Cp
        H = 0.5 * (H + H.conj().T)
        w, V = np.linalg.eigh(H)
        v, lam = V[:, 0], w[0]
        # dL = sum_i g_i Im(dv_i/v_i) - (sum_i g_i) Im(dv_r/v_r) = Im(wv^T dv)
        wv = np.zeros(N, dtype=np.complex128)
        for i in range(N):
            if i != ref:
                wv[i] = g[i, p] / v[i]
        wv[ref] = -(g[:, p].sum() - g[ref, p]) / v[ref]
        u = 1j * np.conj(wv)  # Im(wv^T dv) = Re(u^H dv)
        y = np.zeros(N, dtype=np.complex128)  # (H - lam I)^+ u
        for k in range(1, N):
            y += V[:, k] * (np.vdot(V[:, k], u) / (w[k] - lam))
        Hbar = -np.outer(y, np.conj(v))
        Hbar = 0.5 * (Hbar + Hbar.conj().T)  # dH is Hermitian
        if flags[p] == FLAG_EMI:
            Kbar = np.real(np.conj(Hbar) * Cp)
            Gbar = -Gi @ Kbar @ Gi
            with np.errstate(all="ignore"):
                unit = np.where(G > 0, Cp / G, 0)
            Cbar = Hbar * Gi + Gbar * unit
        else:
            Cbar = -Hbar
        Abar = Cbar / s
        t = np.real(np.conj(Cbar) * Cp)
        Abar[np.arange(N), np.arange(N)] -= 0.5 * (t.sum(axis=1) + t.sum(axis=0)) / d[p]
        S[p] = Abar + Abar.conj().T
    for b, (dy, dx) in enumerate(offs):
        qy, qx = cy[oy] + dy, cx[ox] + dx
        use = bits[:, b] & (qy >= 0) & (qy < R) & (qx >= 0) & (qx < Cc)
        for p in np.nonzero(use)[0]:
            grad[:, qy[p], qx[p]] += S[p] @ z[:, qy[p], qx[p]]
    return grad


# --------------------------------------------------------------------------
# compressed SLC (Sec. 2.2; reading R7)
# --------------------------------------------------------------------------
def compress(stack, first_real, phasors, window):
    """kappa(p) = sum_{i >= first_real} conj(zeta_i(block(p))) z_i(p).

    stack [N, R, C]; phasors [N, oR, oC] (unit modulus).  Returns complex128
    [R, C]."""
    z = np.asarray(stack).astype(np.complex128)
    N, R, C = z.shape
    hx, hy, sx, sy = window
    oR, oC = output_grid(R, C, window)
    by = np.minimum(np.arange(R) // sy, oR - 1)
    bx = np.minimum(np.arange(C) // sx, oC - 1)
    ph = np.asarray(phasors).astype(np.complex128).reshape(N, oR, oC)
    kappa = np.zeros((R, C), dtype=np.complex128)
    for i in range(first_real, N):
        kappa += np.conj(ph[i][by][:, bx]) * z[i]
    return kappa


# --------------------------------------------------------------------------
# single mini-stack and sequential driver (Sec. 2.2 proposed approach, Fig. 1)
# --------------------------------------------------------------------------
def link_ministack(stack, first_real, window, alpha, ref, n_eff=None,
                   stats=None, method="emi"):
    """One mini-stack through the whole path: stats -> GLRT -> coherence ->
    phase linking -> compressed SLC.  Returns a dict of every intermediate."""
    z = np.asarray(stack)
    N, R, C = z.shape
    if stats is None:
        stats = amplitude_stats(z[first_real:])
    mean, var = stats
    n = (N - first_real) if n_eff is None else n_eff
    mask, count, band = shp_select(mean, var, n, window, alpha)
    Cm, valid = coherence(z, mask, window)
    pl = phase_link(Cm, ref=ref, method=method, valid=valid)
    oR, oC = output_grid(R, C, window)
    ph = pl["phasor"].reshape(N, oR, oC)
    kappa = compress(z, first_real, ph, window)
    return {"mean": mean, "var": var, "mask": mask, "count": count, "band": band,
            "coh": Cm, "valid": valid, "link": pl, "phasor": ph, "kappa": kappa}


def sequential(batches, K, window, alpha, method="emi", reference="compressed", decay=1.0):
    """Mini-stack reference scheme of Sec. 2.2 (Fig. 1): mini-stack k is
    [kappa_{k-K} .. kappa_{k-1} | M new SLCs]; its reference is the most
    recent compressed SLC (index 0 for the first mini-stack); earlier batches
    are never re-estimated.  Returns per mini-stack the phasors of its real
    SLCs and its compressed SLC.

    reference="last" forms each compressed SLC with the phasors re-referenced
    to the last real SLC of its mini-stack, so the next mini-stack is linked
    relative to that date (supplement, "Compressed SLC strategy for separate
    batched processing").  decay < 1 weights the statistics of the mini-stack
    of age a (0 = the current one) by M decay^a instead of M (Sec. 3.1: an
    exponential decay that prioritises recent observations), and n_eff is the
    sum of the weights (reading R18)."""
    kappas, groups, out = [], [], []
    for k, znew in enumerate(batches):
        znew = np.asarray(znew)
        M = znew.shape[0]
        groups.append(amplitude_stats(znew) + (M,))
        keep = groups[-(K + 1):]
        wts = [g[2] * decay ** (len(keep) - 1 - j) for j, g in enumerate(keep)]
        mean, var = merge_amplitude_stats([g[0] for g in keep], [g[1] for g in keep], wts)
        n_eff = float(sum(wts))
        comp = kappas[-K:] if K > 0 else []
        stack = np.concatenate([np.stack(comp)] + [znew]) if comp else znew
        ref = len(comp) - 1 if comp else 0
        res = link_ministack(stack, len(comp), window, alpha, ref, n_eff=n_eff,
                             stats=(mean, var), method=method)
        kappa = res["kappa"]
        if reference == "last":
            rot = res["phasor"] * np.conj(res["phasor"][-1])[None]
            kappa = compress(stack, len(comp), rot, window)
        kappas.append(kappa)
        out.append({"phasor": res["phasor"][len(comp):], "kappa": kappa,
                    "n_comp": len(comp), "ref": ref, "mask": res["mask"], "n_eff": n_eff,
                    "flag": res["link"]["flag"], "cond": res["link"]["cond"],
                    "coh": res["coh"], "mean": mean, "var": var})
    return out


def wrap(x):
    """Wrap angles to (-pi, pi]."""
    return np.angle(np.exp(1j * np.asarray(x)))

