"""Plain FP64 CPU oracle for the products built on the linked phases.

TEST INFRASTRUCTURE ONLY.  Like plink_oracle, only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; it shares no code with the GPU library.

Source: Staniewicz et al., "Near-Real-Time InSAR Phase Estimation for
Large-Scale Surface Displacement Monitoring" (arXiv 2511.12051):

* temporal coherence gamma_t (Sec. 3.3, eq. temporal-coherence);
* phase cosine similarity gamma_s (Sec. 3.3, eq. phase-cosine-sim) over the
  nearest-k interferogram network of Sec. 3.4;
* persistent-scatterer selection by the amplitude dispersion D_A (Sec. 3.1,
  threshold of Sec. 4) and the regridding of PS and DS phases to the output
  grid (supplement, "Regridding PS and DS to 30 m resolution");
* the L1 network inversion (Sec. 3.5, eq. l1-min) by ADMM (Appendix A).

Readings where the paper is silent (each listed in the design doc):

* R14 gamma_t: phi_ik is the phase of C_ik (the multilooked interferogram of
  images i and k, z z^H convention so it estimates phi_i - phi_k) and
  hat-phi_ik = hat-phi_i - hat-phi_k; N_ifg = N(N-1)/2 over the N images of the
  linked stack.  A zero C_ik has phase 0.  gamma_t = 1 for N = 1 (no
  interferogram), 0 for an invalid pixel.
* R15 gamma_s: the window is the disk of radius r output pixels around p
  (p itself excluded, pixels outside the grid or invalid excluded); the
  interferograms are the nearest-k network, pairs (a, b) with
  1 <= b - a <= k; s = mean over them of cos((phi_a - phi_b)(p) -
  (phi_a - phi_b)(q)); the median of an even count is the mean of the two
  middle values; a pixel without neighbours, or invalid, gets 0.
* R16 PS: D_A = sigma_A / mu_A from the same amplitude statistics as the
  GLRT; a pixel is a PS iff mu_A > 0 and D_A <= threshold.  Its phase for
  image i is the single-reference phase arg(z_i conj(z_ref)).  The block of
  an output pixel is the set of full-resolution pixels that map to it (the
  block mapping of the compressed SLC, reading R7); among several PS the one
  of lowest D_A wins, ties to the first in row-major order.
* R17 ADMM: A is the incidence matrix of the network with the first date as
  reference (row of pair (a, b): +1 at date b, -1 at date a, column d - 1 for
  date d >= 1); z^0 = u^0 = 0; a fixed number of iterations and a fixed rho.
"""
from __future__ import annotations

import numpy as np

FLAG_INVALID = 2


# --------------------------------------------------------------------------
# temporal coherence (Sec. 3.3, eq. temporal-coherence; reading R14)
# --------------------------------------------------------------------------
def temporal_coherence(Cmat, phase, flags=None):
    """gamma_t of each pixel: Cmat complex [P, N, N], phase [N, P] linked
    phases (radians), flags [P] (FLAG_INVALID pixels get 0)."""
    Cm = np.asarray(Cmat, dtype=np.complex128)
    ph = np.asarray(phase, dtype=np.float64)
    P, N, _ = Cm.shape
    if N < 2:
        out = np.ones(P)
    else:
        acc = np.zeros(P, dtype=np.complex128)
        for i in range(N):
            for k in range(i + 1, N):
                acc += np.exp(1j * (np.angle(Cm[:, i, k]) - (ph[i] - ph[k])))
        out = np.abs(acc) / (N * (N - 1) / 2)
    if flags is not None:
        out = np.where(np.asarray(flags) == FLAG_INVALID, 0.0, out)
    out[~np.isfinite(out)] = 0.0
    return out


# --------------------------------------------------------------------------
# phase cosine similarity (Sec. 3.3, eq. phase-cosine-sim; reading R15)
# --------------------------------------------------------------------------
def nearest_network(N: int, k: int = 3):
    """Pairs (a, b), a < b, of the nearest-k network (Sec. 3.4), ordered by
    separation d = b - a, then by a."""
    return [(a, a + d) for d in range(1, k + 1) for a in range(N - d)]


def disk_offsets(radius: int):
    """Output-grid offsets (dy, dx) within the radius, the centre excluded."""
    return [(dy, dx) for dy in range(-radius, radius + 1) for dx in range(-radius, radius + 1)
            if (dy, dx) != (0, 0) and dy * dy + dx * dx <= radius * radius]


def phase_similarity(phase, radius, k=3, flags=None):
    """gamma_s [oR, oC] of linked phases phase [N, oR, oC]."""
    ph = np.asarray(phase, dtype=np.float64)
    N, oR, oC = ph.shape
    net = nearest_network(N, k)
    valid = np.ones((oR, oC), bool) if flags is None else (np.asarray(flags).reshape(oR, oC) != FLAG_INVALID)
    ifg = np.stack([ph[a] - ph[b] for a, b in net]) if net else np.zeros((0, oR, oC))
    out = np.zeros((oR, oC))
    offs = disk_offsets(radius)
    for y in range(oR):
        for x in range(oC):
            if not valid[y, x]:
                continue
            sims = []
            for dy, dx in offs:
                qy, qx = y + dy, x + dx
                if 0 <= qy < oR and 0 <= qx < oC and valid[qy, qx]:
                    if net:
                        sims.append(np.mean(np.cos(ifg[:, y, x] - ifg[:, qy, qx])))
                    else:
                        sims.append(1.0)
            if sims:
                out[y, x] = np.median(sims)
    return out


# --------------------------------------------------------------------------
# PS selection and regridding (Sec. 3.1, Sec. 4, supplement; reading R16)
# --------------------------------------------------------------------------
def amplitude_dispersion(mean, var):
    """D_A = sigma_A / mu_A (inf where mu_A <= 0 or not finite)."""
    mean = np.asarray(mean, dtype=np.float64)
    var = np.asarray(var, dtype=np.float64)
    with np.errstate(all="ignore"):
        d = np.sqrt(np.maximum(var, 0.0)) / mean
    return np.where(np.isfinite(d) & (mean > 0), d, np.inf)


def ps_select(mean, var, threshold=0.2):
    """Boolean PS mask [R, C] and D_A [R, C]."""
    d = amplitude_dispersion(mean, var)
    return d <= threshold, d


def regrid_ps_ds(stack, ref, ds_phasor, ps, da, window):
    """Phasors [N, oR, oC] of the output grid: the DS phasors where the
    block holds no PS, else the single-reference phase of the block's PS of
    lowest D_A.  Also returns the flat full-resolution index of the chosen PS
    per output pixel (-1 for DS)."""
    z = np.asarray(stack).astype(np.complex128)
    N, R, C = z.shape
    hx, hy, sx, sy = window
    oR, oC = R // sy, C // sx
    out = np.array(ds_phasor, dtype=np.complex128).reshape(N, oR, oC).copy()
    src = np.full((oR, oC), -1, dtype=np.int64)
    best = np.full((oR, oC), np.inf)
    for y in range(R):
        by = min(y // sy, oR - 1)
        for x in range(C):
            if not ps[y, x]:
                continue
            bx = min(x // sx, oC - 1)
            if da[y, x] < best[by, bx]:  # strict: the first in row-major order keeps a tie
                best[by, bx] = da[y, x]
                src[by, bx] = y * C + x
    for by in range(oR):
        for bx in range(oC):
            if src[by, bx] >= 0:
                y, x = divmod(int(src[by, bx]), C)
                v = z[:, y, x] * np.conj(z[ref, y, x])
                out[:, by, bx] = np.exp(1j * np.angle(v))
                out[ref, by, bx] = 1.0
    return out, src


# --------------------------------------------------------------------------
# L1 network inversion by ADMM (Sec. 3.5, eq. l1-min, Appendix A; R17)
# --------------------------------------------------------------------------
def incidence_matrix(N: int, k: int = 3):
    """A [N_ifg, N - 1] of the nearest-k network, first date as reference."""
    net = nearest_network(N, k)
    A = np.zeros((len(net), N - 1))
    for j, (a, b) in enumerate(net):
        A[j, b - 1] += 1.0
        if a >= 1:
            A[j, a - 1] -= 1.0
    return A


def soft_threshold(a, kappa):
    """S_kappa(a): shrink towards 0 by kappa (Appendix A)."""
    a = np.asarray(a, dtype=np.float64)
    return np.where(a > kappa, a - kappa, np.where(a < -kappa, a + kappa, 0.0))


def l1_invert_admm(A, b, rho=1.0, iters=200):
    """x minimising ||A x - b||_1 for every column of b [N_ifg, P] by the
    ADMM iteration of Appendix A with a Cholesky factor of A^T A shared by
    all pixels.  Returns x [N - 1, P]."""
    from scipy.linalg import cho_factor, cho_solve
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if b.ndim == 1:
        b = b[:, None]
    fac = cho_factor(A.T @ A, lower=True)
    z = np.zeros_like(b)
    u = np.zeros_like(b)
    x = np.zeros((A.shape[1], b.shape[1]))
    for _ in range(iters):
        x = cho_solve(fac, A.T @ (b + z - u))
        Ax = A @ x
        z = soft_threshold(Ax - b + u, 1.0 / rho)
        u = u + Ax - b - z
    return x
