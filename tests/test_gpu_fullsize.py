"""Forward parity at the full workload sizes, in the launch configuration the
benchmark times: the whole GPU path runs on the 2048 x 8192, N = 15 burst and
on the 4096 x 16384, N = 25 scale workload; sampled output pixels (random,
corners and edges) are recomputed by the FP64 oracle one by one on local
crops that hold their whole window.

A crop starts at a multiple of the strides, so the pixel keeps its place in
the crop's output grid, and reaches at least half a window beyond the pixel
centre (or the image edge, which then clips both sides alike): the mask,
coherence and linked phases of the pixel depend on nothing outside it.
Criteria as in the crop parity tests: masks bit-exact except GLRT pairs
within 1e-9 of the threshold, coherence within 1e-4, phases within 1e-3 rad
on well-posed pixels, and the compressed SLC (on the GPU's own phasors)
within 1e-6 of sum |z|.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import plink_oracle as O

pytestmark = pytest.mark.gpu

COH_TOL = 1e-4
PHASE_TOL = 1e-3
N_SAMPLES = 160


def _samples(oR, oC, rng):
    edge = [(0, 0), (0, oC - 1), (oR - 1, 0), (oR - 1, oC - 1), (0, oC // 2), (oR - 1, oC // 3),
            (oR // 2, 0), (oR // 3, oC - 1)]
    rand = [tuple(v) for v in rng.integers(0, [oR, oC], size=(N_SAMPLES - len(edge), 2))]
    return edge + rand


def _crop_for(oy, ox, wl):
    """Stride-aligned crop [y0, y1) x [x0, x1) holding the window of (oy, ox),
    and the pixel's output index inside the crop."""
    hx, hy, sx, sy = wl.window
    ky = -(-(hy + sy) // sy)  # strides above the pixel to cover its window
    kx = -(-(hx + sx) // sx)
    oy0, ox0 = max(0, oy - ky), max(0, ox - kx)
    y0, x0 = oy0 * sy, ox0 * sx
    cy, cx = oy * sy + sy // 2, ox * sx + sx // 2
    # whole strides past the window (or the image edge)
    y1 = min(wl.R, max((oy + 1) * sy, -(-(cy + hy + 1 - y0) // sy) * sy + y0))
    x1 = min(wl.C, max((ox + 1) * sx, -(-(cx + hx + 1 - x0) // sx) * sx + x0))
    if y1 == wl.R or (wl.R - y1) < sy:
        y1 = wl.R
    if x1 == wl.C or (wl.C - x1) < sx:
        x1 = wl.C
    return y0, y1, x0, x1, oy - oy0, ox - ox0


def _run(plink, name, precisions, seed):
    wl = synth.WORKLOADS[name]
    print(f"[fullsize] generating {name} {wl.N}x{wl.R}x{wl.C}", flush=True)
    z = synth.make_stack(wl, seed=seed, device="cuda")
    ref = max(0, wl.n_comp - 1)
    oR, oC = wl.out_shape
    mean, var = plink.amplitude_stats(z[wl.n_comp:].contiguous())
    mask, count = plink.shp_select(mean, var, wl.n_new, wl.window, wl.alpha)
    out = {"mask": mask.cpu().numpy().view(np.uint32), "count": count.cpu().numpy().view(np.uint16)}
    rng = np.random.default_rng(seed)
    samples = _samples(oR, oC, rng)
    for prec in precisions:
        coh = plink.estimate_coherence(z, mask, wl.window, precision=prec)
        ph, lam, flags = plink.phase_link(coh, ref=ref)
        kappa = plink.compress_ministack(z, wl.n_comp, wl.window, ph.view(wl.N, oR, oC))
        idx = torch.tensor([oy * oC + ox for oy, ox in samples], device="cuda")
        out[prec] = {"coh": coh[idx].cpu().numpy(), "ph": ph[:, idx].cpu().numpy(),
                     "flags": flags[idx].cpu().numpy(), "ph_full": ph.view(wl.N, oR, oC),
                     "kappa": kappa}
        del coh
    return wl, z, ref, samples, out


def _check(wl, z, ref, samples, out, precisions):
    hx, hy, sx, sy = wl.window
    oR, oC = wl.out_shape
    nbad_mask, nband = 0, 0
    errs = {p: [] for p in precisions}
    dcoh = {p: 0.0 for p in precisions}
    wp_count = {p: 0 for p in precisions}
    for s, (oy, ox) in enumerate(samples):
        y0, y1, x0, x1, ly, lx = _crop_for(oy, ox, wl)
        zc = z[:, y0:y1, x0:x1].cpu().numpy()
        r = O.link_ministack(zc, wl.n_comp, wl.window, wl.alpha, ref)
        _, _, _, stat = O.shp_select(r["mean"], r["var"], wl.n_new, wl.window, wl.alpha, return_stat=True)
        # mask bits of this pixel, excluding the GLRT band
        gm = O.mask_bits(out["mask"][oy, ox][None, :], wl.window)[0]
        om = O.mask_bits(r["mask"][ly, lx][None, :], wl.window)[0]
        thr = O.glrt_threshold(wl.alpha)
        band = np.abs(stat[ly, lx] - thr) < O.GLRT_BAND
        nband += int(band.sum())
        nbad_mask += int(np.sum((gm != om) & ~band))
        cOR, cOC = O.output_grid(y1 - y0, x1 - x0, wl.window)
        p_loc = ly * cOC + lx
        Co = r["coh"][p_loc]
        for prec in precisions:
            Cg = out[prec]["coh"][s].astype(np.complex128)
            if np.any(band):
                continue  # a band pair may legitimately differ: coherence and phases are not comparable
            d = np.nanmax(np.abs(Cg - Co)) if np.all(np.isfinite(Co)) else 0.0
            dcoh[prec] = max(dcoh[prec], d)
            if out[prec]["flags"][s] != r["link"]["flag"][p_loc] or r["link"]["flag"][p_loc] == O.FLAG_INVALID:
                continue
            sens = O.phase_sensitivity(Co[None], ref=ref)[0]
            if 3.0 * sens * max(d, 1e-6) > PHASE_TOL:
                continue
            wp_count[prec] += 1
            e = np.abs(np.angle(out[prec]["ph"][:, s] * np.conj(r["link"]["phasor"][:, p_loc])))
            errs[prec].append(e.max())
    print(f"[fullsize] {wl.name}: {len(samples)} samples, mask mismatches {nbad_mask}, band pairs {nband}", flush=True)
    assert nbad_mask == 0
    for prec in precisions:
        worst = max(errs[prec]) if errs[prec] else 0.0
        print(f"[fullsize] {wl.name} {prec}: max |dC| {dcoh[prec]:.2e}, well-posed {wp_count[prec]}, "
              f"max phase err {worst:.2e} rad", flush=True)
        assert dcoh[prec] <= COH_TOL
        assert wp_count[prec] >= 0.8 * len(samples)
        assert worst <= PHASE_TOL


def _check_kappa(wl, z, out, prec, rng):
    """Compressed SLC at sampled full-resolution pixels, on the GPU's phasors."""
    hx, hy, sx, sy = wl.window
    oR, oC = wl.out_shape
    ys = rng.integers(0, wl.R, 200)
    xs = rng.integers(0, wl.C, 200)
    ys[:2], xs[:2] = [0, wl.R - 1], [0, wl.C - 1]
    by, bx = np.minimum(ys // sy, oR - 1), np.minimum(xs // sx, oC - 1)
    phf = out[prec]["ph_full"]
    kap = out[prec]["kappa"]
    yi, xi = torch.tensor(ys, device="cuda"), torch.tensor(xs, device="cuda")
    zz = z[:, yi, xi].cpu().numpy().astype(np.complex128)         # [N, S]
    pp = phf[:, torch.tensor(by, device="cuda"), torch.tensor(bx, device="cuda")].cpu().numpy().astype(np.complex128)
    got = kap[yi, xi].cpu().numpy()
    for s in range(len(ys)):
        # the oracle's compress on the one-pixel image holding this sample
        want = O.compress(zz[:, s][:, None, None], wl.n_comp, pp[:, s][:, None, None], (0, 0, 1, 1))[0, 0]
        scale = np.abs(zz[wl.n_comp:, s]).sum()
        assert abs(got[s] - want) <= 1e-6 * scale + 1e-30, (ys[s], xs[s])


@pytest.mark.parametrize("name,precisions,seed", [("burst", ("bf16", "fp32"), 81), ("scale", ("bf16",), 82)])
def test_full_size_sampled_parity(gpu_lib, name, precisions, seed):
    wl, z, ref, samples, out = _run(gpu_lib, name, precisions, seed)
    _check(wl, z, ref, samples, out, precisions)
    _check_kappa(wl, z, out, precisions[0], np.random.default_rng(seed + 1))
    del z, out
    torch.cuda.empty_cache()
