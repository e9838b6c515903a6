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
whose EMI/EVD choice differs between the two sides must have an oracle
minimum LDL^T pivot inside a band around tau: [tau/2, 2 tau] when the GPU
links the oracle's own matrices, [tau/10, 10 tau] end to end (the GPU's C then
differs by up to EPS, which moves the pivots); they are counted, not
compared.
"""
import numpy as np

from oracle import plink_oracle as O

PHASE_TOL = 1e-3
COH_TOL = 1e-4
EPS = {"fp32": 2e-6, "bf16": 1.2e-5}
SAFETY = 3.0
BOUND_SAFETY = 10.0
N_PROBE = 8


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


def check_phases(label, err, sens, flags_gpu, link, prec, dC_pix=None, min_well_posed=1, band=10.0):
    """Asserts the criterion above; err [N, P] wrapped errors, sens [P],
    flags_gpu [P], link the oracle's phase_link result.  Returns counts."""
    e = np.asarray(err).max(axis=0)
    flag_o = np.asarray(link["flag"])
    flags_gpu = np.asarray(flags_gpu).reshape(-1)
    boundary = (link["min_pivot"] > O.TAU_PIVOT / band) & (link["min_pivot"] < band * O.TAU_PIVOT)
    same = flags_gpu == flag_o
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
