"""GPU adjoint of coherence + EMI/EVD linking against the FP64 oracle.

The oracle's adjoint (oracle.phase_link_vjp) is itself pinned to FP64 central
differences and to the phase-screen identity by the CPU tests.  Here the HIP
adjoint is compared with it on the same stack, mask and EMI/EVD flags, with
dL/dphi restricted to well-posed pixels (the criterion of the forward parity
tests): on an ill-posed pixel the FP32 eigenvector, and hence its derivative,
is not resolvable.

Tolerance.  The gradient is a sum over the window of S_p z_q; on well-posed
pixels the FP32 forward resolves the phases to <= 1e-3 rad, and the adjoint's
relative error is bounded by the same rounding amplified by one more factor of
the eigen-gap.  The bars sit at about twice the largest error measured on
these cases: 3e-4 of the largest gradient magnitude per element, and 5e-3
relative on every element above a tenth of it.  The well-posed set is the
forward tests' (tests/phase_parity.py), from the oracle alone.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import plink_oracle as O
from phase_parity import well_posed, sensitivity

pytestmark = pytest.mark.gpu

ABS_TOL = 3e-4   # of max |grad|
REL_TOL = 5e-3   # on elements above 0.1 max |grad|


def _forward(plink, z, wl, ref, method, prec="fp32"):
    mean, var = plink.amplitude_stats(z[wl.n_comp:].contiguous())
    mask, _ = plink.shp_select(mean, var, wl.n_new, wl.window, wl.alpha)
    coh = plink.estimate_coherence(z, mask, wl.window, precision=prec)
    ph, lam, flags = plink.phase_link(coh, ref=ref, method=method)
    return mask, coh, ph, flags


def _well_posed(Cgpu, Corc, ref, method):
    return well_posed(sensitivity(Corc, ref, method), "fp32")


def _compare(g_gpu, g_orc, what):
    scale = np.abs(g_orc).max()
    err = np.abs(g_gpu - g_orc)
    big = np.abs(g_orc) > 0.1 * scale
    rel = (err[big] / np.abs(g_orc[big])).max() if big.any() else 0.0
    print(f"[adjoint] {what}: max|grad| {scale:.3e}, max abs err {err.max():.3e} "
          f"({err.max() / scale:.2e} of max), max rel err on large {rel:.2e}", flush=True)
    assert np.all(np.isfinite(g_gpu))
    assert err.max() <= ABS_TOL * scale
    assert rel <= REL_TOL


@pytest.mark.parametrize("method", ["emi", "evd"])
def test_vjp_matches_oracle(gpu_lib, method):
    plink = gpu_lib
    wl = synth.crop("adjoint", 36, 42)  # N = 20, 15 x 15 window, stride 1: every pixel is an output
    z_cpu = synth.make_stack(wl, seed=21)
    z = z_cpu.cuda()
    ref = 3
    mask, coh, ph, flags = _forward(plink, z, wl, ref, method)
    mask_np = mask.cpu().numpy().view(np.uint32)
    flags_np = flags.cpu().numpy()
    Corc, valid = O.coherence(z_cpu.numpy(), mask_np, wl.window)
    wp = _well_posed(coh.cpu().numpy(), Corc, ref, method) & (flags_np != O.FLAG_INVALID)
    print(f"[adjoint] {method}: {wp.sum()} of {wp.size} pixels well-posed; "
          f"EVD flags {(flags_np == O.FLAG_EVD).sum()}", flush=True)
    assert wp.mean() > 0.8
    rng = np.random.default_rng(5)
    g = rng.standard_normal((wl.N, wp.size)).astype(np.float32) * wp[None, :]
    g_dev = torch.from_numpy(g).cuda()
    grad = plink.phase_link_vjp(z, mask, flags, wl.window, ref, g_dev).cpu().numpy()
    want = O.phase_link_vjp(z_cpu.numpy(), mask_np, wl.window, ref, g.astype(np.float64), flags_np)
    _compare(grad.astype(np.complex128), want, f"{method} 36x42 N=20")


def test_vjp_phase_screen_identity_full_size(gpu_lib):
    """At the full 512 x 512, N = 20 size: a per-image phase screen
    dz_n = j delta_n z_n moves phi_i by exactly delta_i - delta_ref, so for
    every image n, -sum_q Im(conj(grad_nq) z_nq) = sum_p g_np - [n = ref] sum_{p,i} g_ip."""
    plink = gpu_lib
    wl = synth.WORKLOADS["adjoint"]
    z = synth.make_stack(wl, seed=22, device="cuda")
    ref = 0
    mask, coh, ph, flags = _forward(plink, z, wl, ref, "emi")
    P = wl.R * wl.C
    rng = np.random.default_rng(6)
    # a sparse random set of pixels carries dL/dphi; ill-posed ones are dropped
    pick = rng.choice(P, 4000, replace=False)
    zc = z.cpu().numpy()
    mask_np = mask.cpu().numpy().view(np.uint32)
    oy, ox = np.divmod(pick, wl.C)
    Corc, _ = O.coherence(zc, mask_np, wl.window, pixels=np.stack([oy, ox], 1))
    Cg = coh.cpu().numpy()[pick]
    wp = _well_posed(Cg, Corc, ref, "emi") & (flags.cpu().numpy()[pick] != O.FLAG_INVALID)
    pick = pick[wp]
    g = np.zeros((wl.N, P), dtype=np.float32)
    g[:, pick] = rng.standard_normal((wl.N, len(pick))).astype(np.float32)
    grad = plink.phase_link_vjp(z, mask, flags, wl.window, ref, torch.from_numpy(g).cuda())
    c = -(torch.conj(grad) * z).imag.double().sum(dim=(1, 2)).cpu().numpy()
    want = g.astype(np.float64).sum(axis=1)
    want[ref] -= g.astype(np.float64).sum()
    scale = np.abs(g).sum() / wl.N
    err = np.abs(c - want).max()
    print(f"[adjoint] phase screen, {len(pick)} pixels: max |c - want| {err:.3e}, scale {scale:.3e}", flush=True)
    assert err <= 1e-3 * scale


def test_vjp_full_size_sampled(gpu_lib):
    """512 x 512, N = 20 in the launch configuration of the full workload;
    the gradient at sampled input pixels against the oracle on local crops
    (at stride 1 the gradient at q depends only on pixels within 2 h of q)."""
    plink = gpu_lib
    wl = synth.WORKLOADS["adjoint"]
    hx, hy, sx, sy = wl.window
    assert sx == 1 and sy == 1
    z = synth.make_stack(wl, seed=23, device="cuda")
    ref = 0
    mask, coh, ph, flags = _forward(plink, z, wl, ref, "emi")
    zc = z.cpu().numpy()
    mask_np = mask.cpu().numpy().view(np.uint32)
    flags_np = flags.cpu().numpy().reshape(wl.R, wl.C)
    Cg = coh.cpu().numpy().reshape(wl.R, wl.C, wl.N, wl.N)
    rng = np.random.default_rng(7)
    g = rng.standard_normal((wl.N, wl.R, wl.C)).astype(np.float32)
    # samples: corners, edges and random interior pixels
    qs = [(0, 0), (0, wl.C - 1), (wl.R - 1, 0), (wl.R - 1, wl.C - 1), (0, 200), (300, wl.C - 1)]
    qs += [tuple(v) for v in rng.integers(0, [wl.R, wl.C], size=(10, 2))]
    # zero dL/dphi on ill-posed pixels near every sample (oracle sensitivity on the crops)
    crops = []
    for qy, qx in qs:
        y0, y1 = max(0, qy - 2 * hy), min(wl.R, qy + 2 * hy + 1)
        x0, x1 = max(0, qx - 2 * hx), min(wl.C, qx + 2 * hx + 1)
        Corc, _ = O.coherence(zc[:, y0:y1, x0:x1], mask_np[y0:y1, x0:x1], wl.window)
        wp = _well_posed(Cg[y0:y1, x0:x1].reshape(-1, wl.N, wl.N), Corc, ref, "emi")
        wp &= flags_np[y0:y1, x0:x1].ravel() != O.FLAG_INVALID
        g[:, y0:y1, x0:x1] *= wp.reshape(1, y1 - y0, x1 - x0)
        crops.append((qy, qx, y0, y1, x0, x1))
    grad = plink.phase_link_vjp(z, mask, flags, wl.window, ref,
                                torch.from_numpy(g.reshape(wl.N, -1)).cuda()).cpu().numpy()
    got, want = [], []
    for qy, qx, y0, y1, x0, x1 in crops:
        gc = g[:, y0:y1, x0:x1].reshape(wl.N, -1).astype(np.float64)
        o = O.phase_link_vjp(zc[:, y0:y1, x0:x1], mask_np[y0:y1, x0:x1], wl.window, ref, gc,
                             flags_np[y0:y1, x0:x1].ravel())
        want.append(o[:, qy - y0, qx - x0])
        got.append(grad[:, qy, qx])
    _compare(np.array(got).astype(np.complex128), np.array(want), "512x512 N=20 sampled")


def test_autograd_function(gpu_lib):
    plink = gpu_lib
    wl = synth.crop("adjoint", 24, 30)
    z = synth.make_stack(wl, seed=24, device="cuda")
    mean, var = plink.amplitude_stats(z)
    mask, _ = plink.shp_select(mean, var, wl.n_new, wl.window, wl.alpha)
    zz = z.clone().requires_grad_(True)
    phase, flags = plink.PhaseLink.apply(zz, mask, wl.window, 2)
    coh = plink.estimate_coherence(z, mask, wl.window)
    ph, _, fl = plink.phase_link(coh, ref=2)
    oR, oC = wl.out_shape
    assert torch.equal(flags, fl)
    np.testing.assert_allclose(np.exp(1j * phase.detach().cpu().numpy().reshape(wl.N, -1)),
                               ph.cpu().numpy(), atol=2e-6)
    assert torch.all(phase[2] == 0)
    w = torch.randn((wl.N, oR, oC), device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    (phase * w).sum().backward()
    direct = plink.phase_link_vjp(z, mask, flags, wl.window, 2, w.reshape(wl.N, -1).contiguous())
    assert torch.equal(zz.grad, direct)


# ---------------------------------------------------------------- FP64 adjoint
def _fd_case():
    from adjoint_fd import fd_gradient
    wl = synth.crop("adjoint", 36, 36)
    z = synth.make_stack(wl, seed=51)
    zn = z.numpy().astype(np.complex128)
    mean, var = O.amplitude_stats(zn)
    mask, _, _ = O.shp_select(mean, var, wl.n_new, wl.window, wl.alpha)
    Cm, valid = O.coherence(zn, mask, wl.window)
    ref = 2
    flags = O.phase_link(Cm, ref=ref, valid=valid)["flag"]
    rng = np.random.default_rng(52)
    g = rng.normal(size=(wl.N, len(flags)))
    entries = [(int(rng.integers(wl.N)), int(rng.integers(wl.R)), int(rng.integers(wl.C))) for _ in range(64)]
    fd = fd_gradient(zn, mask, wl.window, ref, flags, g, entries)
    return wl, z, mask, flags, ref, g, entries, fd


def test_vjp64_matches_finite_differences(gpu_lib):
    """The differentiation configuration's shape (N = 20, half-window 7 x 7,
    stride 1): the FP64 adjoint against FP64 central differences (h = 1e-6)
    of the oracle at 64 random input pixels, to 1e-6 relative, and against
    the oracle's adjoint element by element.  dL/dphi is rounded to FP32 (the
    entry point's type) on both sides."""
    plink = gpu_lib
    wl, z, mask, flags, ref, g, entries, fd = _fd_case()
    g32 = g.astype(np.float32)
    # the differences above used g in FP64; recompute them with the FP32 values
    from adjoint_fd import fd_gradient
    fd = fd_gradient(z.numpy().astype(np.complex128), mask, wl.window, ref, flags, g32.astype(np.float64), entries)
    grad = plink.phase_link_vjp(z.cuda(), torch.from_numpy(mask.view(np.int32)).cuda(),
                                torch.from_numpy(flags).cuda(), wl.window, ref, torch.from_numpy(g32).cuda(),
                                precision="fp64").cpu().numpy()
    an = np.array([grad[n, y, x] for n, y, x in entries]).astype(np.complex128)
    rel = np.linalg.norm(an - fd) / np.linalg.norm(fd)
    want = O.phase_link_vjp(z.numpy(), mask, wl.window, ref, g32.astype(np.float64), flags)
    d = np.abs(grad.astype(np.complex128) - want).max() / np.abs(want).max()
    print(f"[adjoint] FP64 vs finite differences: {rel:.2e} relative; vs oracle adjoint {d:.2e} of max", flush=True)
    assert rel <= 1e-6
    assert d <= 1e-6  # the complex64 rounding of the output (6e-8) dominates


def test_vjp64_full_size_phase_screen_and_samples(gpu_lib):
    """512 x 512, N = 20: the phase-screen identity over the whole image to
    1e-6 relative (the gradient is rounded to complex64), and sampled input
    pixels against the oracle's adjoint on local crops with dL/dphi on every
    pixel (no well-posed restriction is needed in FP64)."""
    plink = gpu_lib
    wl = synth.WORKLOADS["adjoint"]
    hx, hy, sx, sy = wl.window
    z = synth.make_stack(wl, seed=23, device="cuda")
    ref = 0
    mask, coh, ph, flags = _forward(plink, z, wl, ref, "emi")
    P = wl.R * wl.C
    rng = np.random.default_rng(8)
    # dL/dphi on 4000 random pixels (an EMI pixel whose |C| stops inverting
    # in FP64 would contribute nothing; on a random subset that is unlikely
    # and would show as a failure)
    g = np.zeros((wl.N, P), np.float32)
    pick = rng.choice(P, 4000, replace=False)
    g[:, pick] = rng.standard_normal((wl.N, 4000)).astype(np.float32)
    grad = plink.phase_link_vjp(z, mask, flags, wl.window, ref, torch.from_numpy(g).cuda(), precision="fp64")
    torch.cuda.synchronize()
    c = -(torch.conj(grad.to(torch.complex128)) * z.to(torch.complex128)).imag.sum(dim=(1, 2)).cpu().numpy()
    fl = flags.cpu().numpy()
    gv = g.astype(np.float64) * (fl != O.FLAG_INVALID)[None]
    want = gv.sum(axis=1)
    want[ref] -= gv.sum()
    scale = np.abs(gv).sum() / wl.N
    err = np.abs(c - want).max()
    print(f"[adjoint] FP64 phase screen, full size: max |c - want| {err:.3e}, scale {scale:.3e}", flush=True)
    assert err <= 1e-6 * scale
    g = rng.standard_normal((wl.N, P)).astype(np.float32)
    grad = plink.phase_link_vjp(z, mask, flags, wl.window, ref, torch.from_numpy(g).cuda(), precision="fp64")
    zc = z.cpu().numpy()
    mask_np = mask.cpu().numpy().view(np.uint32)
    flags_np = fl.reshape(wl.R, wl.C)
    gg = g.reshape(wl.N, wl.R, wl.C)
    grad = grad.cpu().numpy()
    worst, scale = 0.0, 0.0
    for qy, qx in [(0, 0), (wl.R - 1, wl.C - 1), (0, 300)] + [tuple(v) for v in rng.integers(0, [wl.R, wl.C], (5, 2))]:
        y0, y1 = max(0, qy - 2 * hy), min(wl.R, qy + 2 * hy + 1)
        x0, x1 = max(0, qx - 2 * hx), min(wl.C, qx + 2 * hx + 1)
        o = O.phase_link_vjp(zc[:, y0:y1, x0:x1], mask_np[y0:y1, x0:x1], wl.window, ref,
                             gg[:, y0:y1, x0:x1].reshape(wl.N, -1).astype(np.float64), flags_np[y0:y1, x0:x1].ravel())
        worst = max(worst, np.abs(grad[:, qy, qx] - o[:, qy - y0, qx - x0]).max())
        scale = max(scale, np.abs(o[:, qy - y0, qx - x0]).max())
    print(f"[adjoint] FP64 sampled full size: max err {worst:.3e} of max |grad| {scale:.3e}", flush=True)
    assert worst <= 1e-6 * scale


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-7), ("fp32", 2e-3)])
def test_uncertainty_propagation_per_slc_phase(gpu_lib, precision, tol):
    """A 0.1-rad phase perturbation of each SLC (one value per image),
    linearised through the adjoint: with J_in(p) = dphi_i(p) / d delta_n =
    -sum_q Im(conj(dphi_i(p)/dz_n(q)) z_n(q)), std(phi_i) = 0.1 sqrt(sum_n J_in^2)
    must be 0.1 sqrt(2) for i != ref and 0 at ref (phi_i moves by
    delta_i - delta_ref exactly).  64 output pixels on a grid 64 pixels apart,
    so that one adjoint call per image i (dL/dphi = 1 at the 64 pixels for
    image i) gives every pixel's row of J from its own window region."""
    plink = gpu_lib
    wl = synth.WORKLOADS["adjoint"]
    hx, hy, _, _ = wl.window
    z = synth.make_stack(wl, seed=24, device="cuda")
    ref = 3
    mask, coh, ph, flags = _forward(plink, z, wl, ref, "emi")
    pts = [(32 + 64 * a, 32 + 64 * b) for a in range(8) for b in range(8)]
    fl = flags.cpu().numpy().reshape(wl.R, wl.C)
    pts = [p for p in pts if fl[p] != O.FLAG_INVALID]
    N = wl.N
    J = np.zeros((len(pts), N, N))
    for i in range(N):
        g = torch.zeros((N, wl.R, wl.C), dtype=torch.float32, device="cuda")
        for (y, x) in pts:
            g[i, y, x] = 1.0
        grad = plink.phase_link_vjp(z, mask, flags, wl.window, ref, g.reshape(N, -1), precision=precision)
        prod = -(torch.conj(grad.to(torch.complex128)) * z.to(torch.complex128)).imag  # [N, R, C]
        for k, (y, x) in enumerate(pts):
            J[k, i] = prod[:, y - 2 * hy:y + 2 * hy + 1, x - 2 * hx:x + 2 * hx + 1].sum(dim=(1, 2)).cpu().numpy()
    std = 0.1 * np.sqrt((J ** 2).sum(axis=2))  # [pixels, N]
    want = np.full(N, 0.1 * np.sqrt(2.0))
    want[ref] = 0.0
    err = np.abs(std - want[None]).max()
    print(f"[adjoint] {precision} uncertainty of {len(pts)} pixels: max |std - closed form| {err:.2e} rad", flush=True)
    assert err <= tol
