"""Phase parity criterion shared by the GPU tests.

Which pixels are compared at the 1e-3 rad bar is decided from the FP64
oracle alone, before the GPU result is looked at:

* sens_p: the oracle's statistical sensitivity of pixel p's linked phases to a
  change of C (rad per unit change of the entries, N_PROBE random Hermitian
  probes), oracle.phase_sensitivity;
* EPS[prec]: a fixed bound on the coherence error of each GPU path, about
  twice the largest per-element error measured on any parity case.  Every
  coherence test asserts that the GPU stays inside it, so the selection
  below cannot be widened by a less accurate kernel;
* pixel p is *well posed* iff SAFETY * sens_p * EPS[prec] <= 1e-3 rad.  There
  its phases must be within 1e-3 rad of the oracle (wrapped).

Every other pixel is still bounded: its error must stay below
BOUND_SAFETY * sens_p * max(EPS[prec], |dC_p|), capped at pi (a bound of pi
or more says nothing, and such pixels are counted as unresolvable).  Pixels
whose EMI/EVD choice differs between the two sides must be ones where the
oracle finds the choice unstable: a change of every entry of |C| by at most
eps moves LDL^T pivot d_k by at most eps |v_k|_1^2 to first order, v_k being
row k of L^-1 (d_k = 1 / (G_k^-1)_kk and d_k G_k^-1 e_k = L_k^-T e_k), so a
flip is possible only where some |d_k - tau| <= 2 eps |v_k|_1^2.  They are
counted, not compared.

EPS: split BF16 keeps 16 significant bits of each operand (x = hi + lo with
|x - hi - lo| <= 2^-16 |x|) and drops lo*lo, so each product carries a
relative error of at most about 3 * 2^-16 and, by Cauchy-Schwarz, the
normalised C at most about 6 * 2^-16 = 9e-5 per element (inside the 1e-4
coherence bar); the largest error measured is 1.6e-5, and EPS is about twice
that.  The FP32 path measures up to 1.1e-6.
"""
import numpy as np

from oracle import plink_oracle as O

PHASE_TOL = 1e-3
COH_TOL = 1e-4
EPS = {"fp32": 2.5e-6, "bf16": 3e-5}
SAFETY = 3.0
BOUND_SAFETY = 10.0
N_PROBE = 8


def _ldl_rows(G):
    """Unpivoted LDL^T of each real symmetric G [P, N, N] (no square roots,
    so it runs through indefinite matrices): returns the pivots d [P, N]
    and L [P, N, N] unit lower triangular."""
    A = np.array(G, dtype=np.float64, copy=True)
    P, N, _ = A.shape
    L = np.broadcast_to(np.eye(N), (P, N, N)).copy()
    d = np.empty((P, N))
    with np.errstate(all="ignore"):
        for k in range(N):
            d[:, k] = A[:, k, k]
            l = A[:, k + 1:, k] / d[:, k, None]
            A[:, k + 1:, k + 1:] -= l[:, :, None] * A[:, None, k, k + 1:]
            L[:, k + 1:, k] = l
    return d, L


def flag_unstable(coh_orc, eps, tau=O.TAU_PIVOT):
    """Pixels whose EMI/EVD choice a change of |C| by eps per entry may flip
    (first order, factor 2 for the rest), or whose pivots are not finite."""
    Cm = np.asarray(coh_orc, dtype=np.complex128)
    P = Cm.shape[0]
    ok = np.all(np.isfinite(Cm.reshape(P, -1)), axis=1)
    G = np.where(ok[:, None, None], np.abs(np.where(ok[:, None, None], Cm, 0)), np.eye(Cm.shape[1]))
    d, L = _ldl_rows(G)
    out = ~np.all(np.isfinite(d), axis=1)
    good = ~out
    if good.any():
        with np.errstate(all="ignore"):
            Li = np.linalg.inv(L[good])
        s = np.abs(Li).sum(axis=2) ** 2  # |v_k|_1^2, row k of L^-1
        near = np.abs(d[good] - tau) <= 2.0 * eps * s
        out[good] = np.any(near | ~np.isfinite(s), axis=1)
    return out & ok


def sensitivity(coh, ref, method="emi"):
    return O.phase_sensitivity(coh, ref=ref, method=method, n_probe=N_PROBE)


def well_posed(sens, prec):
    return SAFETY * np.asarray(sens) * EPS[prec] <= PHASE_TOL


def coherence_error(coh_gpu, coh_orc):
    """Per-pixel max |dC| over finite oracle matrices (0 where the oracle's
    matrix is invalid), and the overall maximum."""
    P = coh_orc.shape[0]
    d = np.abs(np.asarray(coh_gpu).astype(np.complex128) - coh_orc).reshape(P, -1)
    ok = np.all(np.isfinite(coh_orc.reshape(P, -1)), axis=1)
    d = np.where(ok[:, None], d, 0.0)
    d = np.where(np.isfinite(d), d, np.inf)
    dp = d.max(axis=1)
    return dp, float(dp.max()) if P else 0.0


def phase_errors(ph_gpu, ph_orc):
    """Wrapped phase differences [N, P] of two phasor arrays."""
    return np.abs(np.angle(np.asarray(ph_gpu).astype(np.complex128) * np.conj(ph_orc)))


def check_phases(label, err, sens, flags_gpu, link, prec, coh_orc, dC_pix=None, min_well_posed=1, eps=None):
    """Asserts the criterion above; err [N, P] wrapped errors, sens [P],
    flags_gpu [P], link the oracle's phase_link result, coh_orc the oracle's
    matrices (for the flag-stability test, with eps, default EPS[prec]).
    Returns counts."""
    e = np.asarray(err).max(axis=0)
    flag_o = np.asarray(link["flag"])
    flags_gpu = np.asarray(flags_gpu).reshape(-1)
    same = flags_gpu == flag_o
    boundary = flag_unstable(coh_orc, EPS[prec] if eps is None else eps) if not same.all() else same
    assert np.all(same | boundary), f"{label}: {int((~same & ~boundary).sum())} EMI/EVD/invalid flags differ"
    valid = same & (flag_o != O.FLAG_INVALID)
    wp = valid & well_posed(sens, prec)
    worst = float(e[wp].max()) if wp.any() else 0.0
    eps_p = EPS[prec] if dC_pix is None else np.maximum(EPS[prec], dC_pix)
    bound = BOUND_SAFETY * np.asarray(sens) * eps_p
    rest = valid & ~wp & np.isfinite(sens) & (bound < np.pi)
    unres = valid & ~wp & ~rest
    ratio = e[rest] / bound[rest] if rest.any() else np.zeros(0)
    out = dict(pixels=int(e.size), well_posed=int(wp.sum()), bounded=int(rest.sum()),
               unresolvable=int(unres.sum()), flag_boundary=int((~same).sum()), max_err=worst,
               max_bound_ratio=float(ratio.max()) if ratio.size else 0.0,
               p99_err_all_valid=float(np.percentile(e[valid], 99)) if valid.any() else 0.0)
    print(f"[parity] {label} {prec}: " + ", ".join(f"{k} {v:.3g}" if isinstance(v, float) else f"{k} {v}"
                                                     for k, v in out.items()), flush=True)
    assert wp.sum() >= min_well_posed, f"{label}: only {int(wp.sum())} well-posed pixels"
    assert worst <= PHASE_TOL, f"{label}: well-posed phase error {worst:.3e} rad"
    assert np.all(ratio <= 1.0), f"{label}: {int((ratio > 1).sum())} pixels above their error bound"
    return out
