"""Forward parity at the full workload sizes, in the launch configuration the
benchmark times: the whole GPU path runs on the 2048 x 8192, N = 15 burst and
on the 4096 x 16384, N = 25 scale workload; sampled output pixels (random,
corners and edges) are recomputed by the FP64 oracle one by one on local
crops that hold their whole window.

A crop starts at a multiple of the strides, so the pixel keeps its place in
the crop's output grid, and reaches at least half a window beyond the pixel
centre (or the image edge, which then clips both sides alike): the mask,
coherence and linked phases of the pixel depend on nothing outside it.
Criteria as in the crop parity tests (tests/phase_parity.py): masks
bit-exact except GLRT pairs within 1e-9 of the threshold, coherence within
1e-4 and within the fixed per-precision bound EPS, phases within 1e-3 rad on
the pixels the oracle marks well posed and within a per-pixel bound on the
rest, and the compressed SLC (on the GPU's own phasors) within 1e-6 of
sum |z|.

Besides the samples: the SHP masks of the whole 2048 x 8192 burst against the
oracle's, and every output pixel of crops of more than 20,000 output pixels
of both workloads, in both precisions.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import plink_oracle as O
from phase_parity import COH_TOL, EPS, check_phases, coherence_error, phase_errors, sensitivity

pytestmark = pytest.mark.gpu

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
    oR, oC = wl.out_shape
    nbad_mask, nband, band_px = 0, 0, 0
    thr = O.glrt_threshold(wl.alpha)
    keep, Co_all, link = [], [], {"flag": [], "min_pivot": [], "phasor": []}
    for s, (oy, ox) in enumerate(samples):
        y0, y1, x0, x1, ly, lx = _crop_for(oy, ox, wl)
        zc = z[:, y0:y1, x0:x1].cpu().numpy()
        r = O.link_ministack(zc, wl.n_comp, wl.window, wl.alpha, ref)
        _, _, _, stat = O.shp_select(r["mean"], r["var"], wl.n_new, wl.window, wl.alpha, return_stat=True)
        # mask bits of this pixel, excluding the GLRT band
        gm = O.mask_bits(out["mask"][oy, ox][None, :], wl.window)[0]
        om = O.mask_bits(r["mask"][ly, lx][None, :], wl.window)[0]
        band = np.abs(stat[ly, lx] - thr) < O.GLRT_BAND
        nband += int(band.sum())
        nbad_mask += int(np.sum((gm != om) & ~band))
        if np.any(band):
            band_px += 1
            continue  # a band pair may legitimately differ: coherence and phases are not comparable
        cOR, cOC = O.output_grid(y1 - y0, x1 - x0, wl.window)
        p_loc = ly * cOC + lx
        keep.append(s)
        Co_all.append(r["coh"][p_loc])
        for k in link:
            link[k].append(r["link"][k][..., p_loc])
    print(f"[fullsize] {wl.name}: {len(samples)} samples, mask mismatches {nbad_mask}, band pairs {nband} "
          f"in {band_px} pixels", flush=True)
    assert nbad_mask == 0
    Co_all = np.array(Co_all)
    link = {"flag": np.array(link["flag"]), "min_pivot": np.array(link["min_pivot"]),
            "phasor": np.array(link["phasor"]).T}
    sens = sensitivity(Co_all, ref)
    for prec in precisions:
        Cg = out[prec]["coh"][keep]
        dC, dmax = coherence_error(Cg, Co_all)
        print(f"[fullsize] {wl.name} {prec}: max |dC| {dmax:.2e}", flush=True)
        assert dmax <= min(COH_TOL, EPS[prec])
        err = phase_errors(out[prec]["ph"][:, keep], link["phasor"])
        check_phases(f"{wl.name} full size, {len(keep)} samples", err, sens, out[prec]["flags"][keep], link,
                     prec, Co_all, dC_pix=dC, min_well_posed=len(keep) // 10)


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


@pytest.mark.parametrize("name,precisions,seed", [("burst", ("bf16", "fp32"), 81), ("scale", ("bf16", "fp32"), 82)])
def test_full_size_sampled_parity(gpu_lib, name, precisions, seed):
    wl, z, ref, samples, out = _run(gpu_lib, name, precisions, seed)
    _check(wl, z, ref, samples, out, precisions)
    _check_kappa(wl, z, out, precisions[0], np.random.default_rng(seed + 1))
    del z, out
    torch.cuda.empty_cache()


def test_full_size_masks_burst(gpu_lib):
    """Every SHP mask of the 2048 x 8192 burst (930,930 output pixels x 253
    window pairs) against the oracle's, bit-exact outside the GLRT band; the
    amplitude statistics feeding them within 1e-13 / 1e-10."""
    plink = gpu_lib
    wl = synth.WORKLOADS["burst"]
    z = synth.make_stack(wl, seed=83, device="cuda")
    mean, var = plink.amplitude_stats(z)
    cnt = plink.new_counters()
    mask, count = plink.shp_select(mean, var, wl.n_new, wl.window, wl.alpha, counters=cnt)
    mask = mask.cpu().numpy().view(np.uint32)
    zc = z.cpu().numpy()
    del z
    torch.cuda.empty_cache()
    print("[fullsize] oracle statistics and masks of the 2048x8192 burst", flush=True)
    mo, vo = O.amplitude_stats(zc)
    del zc
    np.testing.assert_allclose(mean.cpu().numpy(), mo, rtol=1e-13)
    np.testing.assert_allclose(var.cpu().numpy(), vo, rtol=1e-10, atol=1e-15 * mo.max() ** 2)
    om, ocount, band, stat = O.shp_select(mo, vo, wl.n_new, wl.window, wl.alpha, return_stat=True)
    inband = np.abs(stat - O.glrt_threshold(wl.alpha)) < O.GLRT_BAND
    del stat
    diff = (O.mask_bits(mask, wl.window) != O.mask_bits(om, wl.window)) & ~inband
    print(f"[fullsize] burst masks: {mask.shape[0] * mask.shape[1]} pixels, band pairs oracle {band} "
          f"gpu {int(cnt[0].item())}, mismatches outside the band {int(diff.sum())}", flush=True)
    assert not diff.any()
    ok = ~inband.any(-1)
    np.testing.assert_array_equal(count.cpu().numpy().view(np.uint16)[ok], ocount[ok])


@pytest.mark.parametrize("name,R,C,seed", [("burst", 288, 1536, 84), ("scale", 288, 1280, 85)])
def test_large_crop_every_pixel(gpu_lib, name, R, C, seed):
    """Every output pixel of a crop with more than 20,000 of them (96 x 256 at
    N = 15, 96 x 213 at N = 25), both precisions, in the single-call launch
    configuration of the full workload."""
    plink = gpu_lib
    wl = synth.crop(name, R, C)
    z = synth.make_stack(wl, seed=seed)
    ref = max(0, wl.n_comp - 1)
    print(f"[fullsize] oracle on the {R}x{C} {name} crop", flush=True)
    orc = O.link_ministack(z.numpy(), wl.n_comp, wl.window, wl.alpha, ref)
    _, _, nband, stat = O.shp_select(orc["mean"], orc["var"], wl.n_new, wl.window, wl.alpha, return_stat=True)
    inband = (np.abs(stat - O.glrt_threshold(wl.alpha)) < O.GLRT_BAND).any(-1).reshape(-1)
    sens = sensitivity(orc["coh"], ref)
    P = len(sens)
    assert P > 20000
    zc = z.cuda()
    mean, var = plink.amplitude_stats(zc[wl.n_comp:].contiguous())
    mask, _ = plink.shp_select(mean, var, wl.n_new, wl.window, wl.alpha)
    diff = (O.mask_bits(mask.cpu().numpy().view(np.uint32), wl.window) != O.mask_bits(orc["mask"], wl.window))
    assert not (diff.reshape(P, -1) & ~inband[:, None]).any()
    print(f"[fullsize] {name} crop: {P} output pixels, {nband} band pairs in {int(inband.sum())} pixels",
          flush=True)
    keep = ~inband
    for prec in ("bf16", "fp32"):
        coh = plink.estimate_coherence(zc, mask, wl.window, precision=prec)
        ph, lam, flags = plink.phase_link(coh, ref=ref)
        dC, dmax = coherence_error(coh.cpu().numpy()[keep], orc["coh"][keep])
        print(f"[fullsize] {name} crop {prec}: max |dC| {dmax:.2e}", flush=True)
        assert dmax <= min(COH_TOL, EPS[prec])
        link = {k: orc["link"][k][..., keep] for k in ("flag", "min_pivot", "phasor")}
        err = phase_errors(ph.cpu().numpy()[:, keep], link["phasor"])
        check_phases(f"{name} {R}x{C} crop", err, sens[keep], flags.cpu().numpy()[keep], link, prec,
                     orc["coh"][keep], dC_pix=dC, min_well_posed=int(keep.sum()) // 10)
