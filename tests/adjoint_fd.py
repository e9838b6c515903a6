"""FP64 central finite differences of L = sum_p sum_i g_i(p) phi_i(p) through
the oracle, for the adjoint tests: perturbing z_n(q) moves only the output
pixels whose window holds q, so each difference re-links just those."""
import numpy as np

from oracle import plink_oracle as O


def affected_pixels(q, shape, window):
    """Output pixels (oy, ox) whose window holds input pixel q = (y, x)."""
    R, C = shape
    hx, hy, sx, sy = window
    cy, cx = O.output_centres(R, C, window)
    oy = np.nonzero(np.abs(cy - q[0]) <= hy)[0]
    ox = np.nonzero(np.abs(cx - q[1]) <= hx)[0]
    return np.array([(a, b) for a in oy for b in ox])


def fd_gradient(z, mask, window, ref, flags, g, entries, h=1e-6):
    """dL/dRe z + j dL/dIm z at entries [(n, y, x)], central differences with
    step h; g [N, P] is dL/dphi, flags [P] the EMI/EVD choice held fixed."""
    z = np.asarray(z).astype(np.complex128)
    N, R, C = z.shape
    oR, oC = O.output_grid(R, C, window)
    out = np.zeros(len(entries), complex)
    for k, (n, y, x) in enumerate(entries):
        pix = affected_pixels((y, x), (R, C), window)
        idx = pix[:, 0] * oC + pix[:, 1]
        gp = np.asarray(g)[:, idx]
        fl = np.asarray(flags)[idx]
        for unit in (1.0, 1j):
            zp, zm = z.copy(), z.copy()
            zp[n, y, x] += h * unit
            zm[n, y, x] -= h * unit
            lp = np.sum(gp * O.link_phases_fixed(zp, mask, window, ref, fl, pixels=pix))
            lm = np.sum(gp * O.link_phases_fixed(zm, mask, window, ref, fl, pixels=pix))
            d = (lp - lm) / (2 * h)
            out[k] += d if unit == 1.0 else 1j * d
    return out
