"""GPU parity of the products built on the linked phases and of the fused
entry point, against the FP64 oracle (oracle/plink_oracle.py and
oracle/products.py):

* temporal coherence gamma_t from the linking epilogue;
* fused coherence + linking (bands through a bounded buffer): bit-identical
  to the two-step path above 16 images, and to itself for any band height;
* the counters report and its iteration histogram;
* PS selection by D_A and PS/DS regridding;
* phase cosine similarity gamma_s;
* L1 network inversion by ADMM;
* the sequential driver's last-per-ministack reference and exponential
  statistics weights.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import plink_oracle as O
from oracle import products as Q
from phase_parity import EPS, check_phases, coherence_error, phase_errors, sensitivity

pytestmark = pytest.mark.gpu

CROPS = {"burst": ("burst", 192, 390, 12), "scale": ("scale", 99, 384, 13)}
_cache = {}


def _crop(name):
    if name not in _cache:
        wl_name, R, C, seed = CROPS[name]
        wl = synth.crop(wl_name, R, C)
        z = synth.make_stack(wl, seed=seed)
        ref = max(0, wl.n_comp - 1)
        orc = O.link_ministack(z.numpy(), wl.n_comp, wl.window, wl.alpha, ref)
        _cache[name] = (wl, z, ref, orc)
    return _cache[name]


def _mask(plink, wl, zc):
    mean, var = plink.amplitude_stats(zc[wl.n_comp:].contiguous())
    mask, _ = plink.shp_select(mean, var, wl.n_new, wl.window, wl.alpha)
    return mean, var, mask


# ---------------------------------------------------------------- temporal coherence
@pytest.mark.parametrize("name", list(CROPS))
def test_temporal_coherence_epilogue(gpu_lib, name):
    """gamma_t of the linking kernel (fed the oracle's matrices in complex64)
    against the oracle's gamma_t of the same matrices and the GPU's phases
    (the arithmetic alone: FP32 sums of N(N-1)/2 unit phasors, 1e-5), and
    against the oracle's own gamma_t within the Lipschitz bound
    |d gamma_t| <= max_(i,k) |d(phi_i - phi_k)| <= 2 max |d phi|."""
    wl, z, ref, orc = _crop(name)
    C64 = orc["coh"].astype(np.complex64)
    ph, lam, flags, phase, tcoh = gpu_lib.phase_link(torch.from_numpy(C64).cuda(), ref=ref, want_phase=True,
                                                     want_tcoh=True)
    tcoh, phase, flags = tcoh.cpu().numpy(), phase.cpu().numpy().astype(np.float64), flags.cpu().numpy()
    same = (flags == orc["link"]["flag"]) & (flags != O.FLAG_INVALID)
    want = Q.temporal_coherence(C64.astype(np.complex128), phase, flags)
    d = np.abs(tcoh - want)
    print(f"[products] {name}: gamma_t arithmetic max {d.max():.2e}, mean gamma_t {tcoh[same].mean():.3f}")
    assert d.max() <= 1e-5
    g_orc = Q.temporal_coherence(orc["coh"], orc["link"]["phase"], orc["link"]["flag"])
    dphi = np.abs(O.wrap(phase - orc["link"]["phase"])).max(axis=0)
    assert np.all(np.abs(tcoh - g_orc)[same] <= 2 * dphi[same] + 1e-5)
    assert np.all(tcoh[flags == O.FLAG_INVALID] == 0)
    assert np.all((tcoh >= 0) & (tcoh <= 1 + 1e-6))


def test_temporal_coherence_two_images_and_noise_free(gpu_lib):
    rng = np.random.default_rng(40)
    P = 500
    g = rng.uniform(0.05, 0.99, P)
    th = rng.uniform(-np.pi, np.pi, P)
    Cm = np.zeros((P, 2, 2), np.complex64)
    Cm[:, 0, 0] = Cm[:, 1, 1] = 1
    Cm[:, 1, 0] = g * np.exp(1j * th)
    Cm[:, 0, 1] = np.conj(Cm[:, 1, 0])
    t = gpu_lib.phase_link(torch.from_numpy(Cm).cuda(), want_tcoh=True)[3].cpu().numpy()
    np.testing.assert_allclose(t, 1.0, atol=1e-6)
    # noise-free model matrices C = Phi Gamma Phi^H, N = 25 (two rows per lane)
    N = 25
    tt = np.arange(N)
    G = 0.7 * np.exp(-np.abs(tt[:, None] - tt[None, :]) / 5.0) + 0.1
    np.fill_diagonal(G, 1.0)
    phi = rng.uniform(-np.pi, np.pi, (200, N))
    Cm = (np.exp(1j * phi)[:, :, None] * G[None] * np.exp(-1j * phi)[:, None, :]).astype(np.complex64)
    t = gpu_lib.phase_link(torch.from_numpy(Cm).cuda(), ref=7, want_tcoh=True)[3].cpu().numpy()
    np.testing.assert_allclose(t, 1.0, atol=2e-5)


# ---------------------------------------------------------------- fused forward
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("name", list(CROPS))
def test_fused_against_two_step_and_oracle(gpu_lib, name, prec):
    """Bands of 1, 5 and all output rows give bit-identical results (the
    same kernels on the same pixels); above 16 images the fused path is also
    bit-identical to estimate_coherence + phase_link (both read C's upper
    triangle); at every N it meets the oracle by the shared criterion."""
    plink = gpu_lib
    wl, z, ref, orc = _crop(name)
    zc = z.cuda()
    mean, var, mask = _mask(plink, wl, zc)
    row, full = plink.phase_link_fused_workspace(wl.N, wl.R, wl.C, wl.window)
    outs = []
    for rows in (1, 5, 10 ** 6):
        ws = torch.empty((min(full, rows * row),), dtype=torch.uint8, device="cuda")
        outs.append(plink.phase_link_fused(zc, mask, wl.window, ref, prec, want_phase=True, want_tcoh=True,
                                           workspace=ws))
    torch.cuda.synchronize()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert torch.equal(a, b)
    coh = plink.estimate_coherence(zc, mask, wl.window, precision=prec)
    two = plink.phase_link(coh, ref=ref, want_phase=True, want_tcoh=True)
    if wl.N > 16:
        for a, b in zip(outs[0], two):
            assert torch.equal(a, b)
    ph, lam, flags, phase, tcoh = (t.cpu().numpy() for t in outs[0])
    dC, _ = coherence_error(coh.cpu().numpy(), orc["coh"])
    err = phase_errors(ph, orc["link"]["phasor"])
    check_phases(f"fused {name}", err, sensitivity(orc["coh"], ref), flags, orc["link"], prec, orc["coh"],
                 dC_pix=dC, min_well_posed=len(dC) // 10)
    assert np.array_equal(phase[ref], np.zeros_like(phase[ref]))


def test_counters_report_histogram(gpu_lib):
    plink = gpu_lib
    wl, z, ref, orc = _crop("scale")
    zc = z.cuda()
    mean, var, mask = _mask(plink, wl, zc)
    cnt = plink.new_counters()
    ph, lam, flags = plink.phase_link_fused(zc, mask, wl.window, ref, "bf16", counters=cnt)
    rep = plink.sync_report(cnt)
    valid = int((flags != O.FLAG_INVALID).sum().item())
    print(f"[products] report: {rep}")
    assert sum(rep["iter_hist"]) == valid
    assert sum(b * n for b, n in enumerate(rep["iter_hist"][:15])) + 15 * rep["iter_hist"][15] <= rep["iterations"]
    assert rep["evd_fallbacks"] == int((flags == O.FLAG_EVD).sum().item())


# ---------------------------------------------------------------- PS regridding
def test_ps_selection_and_regridding(gpu_lib):
    """On a burst crop (2/7 of the land pixels are PS at D_A ~ 0.1): the PS
    mask from the GPU statistics equals the oracle's on the same statistics
    except where D_A is within 1e-12 of the threshold; the chosen PS per
    block agrees (or has the same D_A within 1e-12); the regridded phasors
    agree with the oracle's within 1e-6 rad."""
    plink = gpu_lib
    wl, z, ref, orc = _crop("burst")
    zc = z.cuda()
    mean, var, mask = _mask(plink, wl, zc)
    ph, _, _ = plink.phase_link(plink.estimate_coherence(zc, mask, wl.window), ref=ref)
    for thr in (0.2, 0.35):
        out, src, ps = plink.ps_regrid(zc, ref, wl.window, mean, var, ph, threshold=thr)
        m, v = mean.cpu().numpy(), var.cpu().numpy()
        ps_o, da = Q.ps_select(m, v, thr)
        band = np.abs(da - thr) <= 1e-12
        assert np.array_equal(ps.cpu().numpy().astype(bool)[~band], ps_o[~band])
        want, src_o = Q.regrid_ps_ds(z.numpy(), ref, ph.cpu().numpy(), ps_o, da, wl.window)
        src = src.cpu().numpy().reshape(src_o.shape)
        diff = src != src_o
        if diff.any():  # ties within rounding: the same D_A
            a = da.ravel()[src[diff]]
            b = da.ravel()[src_o[diff]]
            assert np.all(np.abs(a - b) <= 1e-12), (a, b)
        keep = ~diff.ravel()
        e = np.abs(np.angle(out.cpu().numpy().astype(np.complex128) * np.conj(want.reshape(wl.N, -1))))
        print(f"[products] regrid thr {thr}: PS {int(ps_o.sum())}, blocks with PS {int((src_o >= 0).sum())} "
              f"of {src_o.size}, max phase diff {e[:, keep].max():.2e}")
        assert (src_o >= 0).sum() > 0 and (src_o < 0).sum() > 0
        assert e[:, keep].max() <= 1e-6


# ---------------------------------------------------------------- phase similarity
@pytest.mark.parametrize("name,radius,k", [("burst", 1, 3), ("burst", 7, 3), ("scale", 3, 1), ("scale", 7, 3)])
def test_phase_similarity(gpu_lib, name, radius, k):
    """gamma_s of the GPU's own phasors against the oracle's gamma_s of the
    same phases: the median is 1-Lipschitz in the similarities, which differ
    by FP32 rounding only, so 1e-5 absolute."""
    plink = gpu_lib
    wl, z, ref, orc = _crop(name)
    zc = z.cuda()
    mean, var, mask = _mask(plink, wl, zc)
    ph, lam, flags = plink.phase_link(plink.estimate_coherence(zc, mask, wl.window), ref=ref)
    flags[::7] = O.FLAG_INVALID  # some invalid neighbours and centres
    g = plink.phase_similarity(ph, wl.out_shape, radius, k, flags=flags).cpu().numpy()
    oR, oC = wl.out_shape
    phase = np.angle(ph.cpu().numpy().astype(np.complex128)).reshape(wl.N, oR, oC)
    want = Q.phase_similarity(phase, radius, k, flags=flags.cpu().numpy().reshape(oR, oC)).ravel()
    d = np.abs(g - want)
    print(f"[products] gamma_s {name} r={radius} k={k}: max diff {d.max():.2e}, median gamma_s {np.median(want):.3f}")
    assert d.max() <= 1e-5


# ---------------------------------------------------------------- L1 inversion
@pytest.mark.parametrize("N,k", [(5, 3), (15, 3), (15, 2), (16, 1), (17, 3), (25, 3), (32, 3)])
def test_network_inversion_l1(gpu_lib, N, k):
    """Synthetic unwrapped phases of the nearest-k network with sparse
    unwrapping errors of whole cycles; 200 ADMM iterations, rho = 1, on both
    sides.  The iteration is non-expansive, so FP32 rounding (about 6e-8 of
    the phase scale 1 + max|b| per step, a few roundings per step) adds up at
    most linearly: 200 steps stay within 1e-4 of that scale."""
    plink = gpu_lib
    rng = np.random.default_rng(500 + N * 10 + k)
    P = 3000
    A = Q.incidence_matrix(N, k)
    x_true = np.cumsum(rng.normal(0, 1.0, (N - 1, P)), axis=0)
    b = A @ x_true + rng.normal(0, 0.05, (A.shape[0], P))
    err_rows = rng.random((A.shape[0], P)) < 0.03
    b = b + err_rows * 2 * np.pi * rng.choice([-1, 1], (A.shape[0], P))
    b32 = b.astype(np.float32)
    x, res = plink.network_invert_l1(torch.from_numpy(b32).cuda(), N, k, rho=1.0, iters=200)
    x, res = x.cpu().numpy(), res.cpu().numpy()
    want = Q.l1_invert_admm(A, b32.astype(np.float64), rho=1.0, iters=200)
    d = np.abs(x - want)
    scale = 1.0 + np.abs(b32).max()
    res_o = np.abs(A @ want - b32).sum(axis=0)
    print(f"[products] ADMM N={N} k={k}: max |dx| {d.max():.2e} (scale {scale:.1f}), "
          f"max residual diff {np.abs(res - res_o).max():.2e}", flush=True)
    assert d.max() <= 1e-4 * scale
    assert np.all(np.abs(res - res_o) <= 1e-4 * scale * A.shape[0])


# ---------------------------------------------------------------- driver options
def test_sequential_last_per_ministack_coherent(gpu_lib):
    """Epoch phases shared by every pixel: with reference="last" mini-stack
    k >= 1 is linked relative to the last date of mini-stack k-1, and every
    compressed SLC carries the phase of its mini-stack's last date."""
    plink = gpu_lib
    rng = np.random.default_rng(41)
    M, K, n, R, C, w = 15, 3, 5, 36, 60, (5, 2, 3, 3)
    phi = np.cumsum(rng.uniform(-1, 1, n * M))
    amp = rng.normal(size=(R, C)) + 1j * rng.normal(size=(R, C))
    z = torch.from_numpy((np.exp(1j * phi)[:, None, None] * amp[None]).astype(np.complex64)).cuda()
    seq = plink.Sequential(R, C, M, K, w, reference="last")
    for k in range(n):
        ph, kap, _ = seq.push(z[k * M:(k + 1) * M].contiguous())
        base = phi[0] if k == 0 else phi[k * M - 1]
        want = np.exp(1j * (phi[k * M:(k + 1) * M] - base))[:, None, None]
        err = np.abs(np.angle(ph.cpu().numpy() * np.conj(want)))
        last = z[(k + 1) * M - 1].cpu().numpy().astype(np.complex128)
        inh = np.abs(np.angle(kap.cpu().numpy().astype(np.complex128) * np.conj(last)))
        print(f"[products] last-per-ministack {k}: max phase err {err.max():.2e}, kappa phase {inh.max():.2e}")
        assert err.max() < 2e-3 and inh.max() < 2e-3
    seq.close()


@pytest.mark.parametrize("decay", [1.0, 0.5])
def test_sequential_weight_decay_masks(gpu_lib, decay):
    """Amplitudes constant within each mini-stack (the oracle pin's pattern,
    tiled over a 9 x 9 grid so that every 3 x 3 window holds it): the
    driver's SHP masks of every mini-stack equal the oracle's sequential
    scheme with the same weights (M decay^age) and n_eff, bit for bit; a
    real stack's masks likewise at decay 0.7."""
    plink = gpu_lib
    rng = np.random.default_rng(42)
    M, K, T = 15, 2, 4
    amp = np.ones((T, 9, 9))
    amp[:, 0::3, 0::3] = 1.6
    amp[0, 0::3, 2::3] = 3.0
    amp[1:3, 2::3, 0::3] = 2.0
    amp[3, 2::3, 2::3] = 3.0
    batches = [(amp[k][None] * np.exp(1j * rng.uniform(-np.pi, np.pi, (M, 9, 9)))).astype(np.complex64)
               for k in range(T)]
    win = (1, 1, 3, 3)
    orc = O.sequential(batches, K, win, 1e-3, decay=decay)
    seq = plink.Sequential(9, 9, M, K, win, weight_decay=decay)
    for k in range(T):
        seq.push(torch.from_numpy(batches[k]).cuda())
        m = seq.last_mask().cpu().numpy().view(np.uint32)
        assert np.array_equal(m, orc[k]["mask"]), (decay, k)
    bits = O.mask_bits(orc[3]["mask"], win)[0, 0]
    assert bits[6] == (decay == 0.5)  # the hand-worked decision of the oracle pin
    seq.close()
    wl = synth.crop("sequential", 96, 198)
    z = synth.make_sequence(wl, seed=43, ministacks=4)
    orc = O.sequential([z[k * M:(k + 1) * M].numpy() for k in range(4)], K, wl.window, wl.alpha, decay=0.7)
    seq = plink.Sequential(wl.R, wl.C, M, K, wl.window, wl.alpha, weight_decay=0.7)
    zc = z.cuda()
    for k in range(4):
        seq.push(zc[k * M:(k + 1) * M].contiguous())
        assert np.array_equal(seq.last_mask().cpu().numpy().view(np.uint32), orc[k]["mask"]), k
    seq.close()
