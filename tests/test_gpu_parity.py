"""GPU parity: every step of the HIP path against the FP64 oracle, element by
element, on seeded synthetic stacks that span several tiles with ragged
edges, plus edge cases.

Tolerances (from the workload descriptions): SHP masks bit-exact except GLRT
tests within 1e-9 of the threshold; coherence within 1e-4 per element (and
within the fixed per-precision bound EPS that the phase criterion assumes);
linked phases within 1e-3 rad (wrapped) on the pixels the oracle alone
marks well posed, and within a per-pixel error bound everywhere else
(tests/phase_parity.py states the criterion).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import plink_oracle as O
from phase_parity import COH_TOL, EPS, PHASE_TOL, check_phases, coherence_error, phase_errors, sensitivity

pytestmark = pytest.mark.gpu


def _wl(name, R=None, C=None):
    return synth.WORKLOADS[name] if R is None else synth.crop(name, R, C)


CASES = {
    "tiny": dict(wl=("tiny",), seed=11),
    "burst-crop": dict(wl=("burst", 192, 390), seed=12),   # 64 x 65 outputs: ragged strips
    "scale-crop": dict(wl=("scale", 99, 384), seed=13),    # N = 25, 33 x 64 outputs
    "adjoint-crop": dict(wl=("adjoint", 80, 88), seed=14),  # N = 20, stride 1, 15x15 window
}


class Case:
    def __init__(self, name):
        spec = CASES[name]
        self.name = name
        self.wl = _wl(*spec["wl"])
        self.seed = spec["seed"]
        self.stack = synth.make_stack(self.wl, seed=self.seed)  # CPU, complex64
        self.z = self.stack.numpy()
        wl = self.wl
        self.ref = max(0, wl.n_comp - 1)
        self.first_real = wl.n_comp
        self.orc = O.link_ministack(self.z, self.first_real, wl.window, wl.alpha, self.ref)
        _, _, _, self.stat = O.shp_select(self.orc["mean"], self.orc["var"], wl.n_new, wl.window,
                                          wl.alpha, return_stat=True)
        self.sens = sensitivity(self.orc["coh"], self.ref)


_cache = {}


def case(name):
    if name not in _cache:
        print(f"[parity] preparing oracle for {name}", flush=True)
        _cache[name] = Case(name)
    return _cache[name]


def gpu_path(plink, c: Case, prec="fp32"):
    wl = c.wl
    z = c.stack.cuda()
    mean, var = plink.amplitude_stats(z[c.first_real:].contiguous())
    cnt = plink.new_counters()
    mask, count = plink.shp_select(mean, var, wl.n_new, wl.window, wl.alpha, counters=cnt)
    coh = plink.estimate_coherence(z, mask, wl.window, precision=prec)
    ph, lam, flags = plink.phase_link(coh, ref=c.ref, counters=cnt)
    oR, oC = wl.out_shape
    kappa = plink.compress_ministack(z, c.first_real, wl.window, ph.view(wl.N, oR, oC))
    torch.cuda.synchronize()
    return dict(mean=mean.cpu().numpy(), var=var.cpu().numpy(),
                mask=mask.cpu().numpy().view(np.uint32), count=count.cpu().numpy().view(np.uint16),
                coh=coh.cpu().numpy(), ph=ph.cpu().numpy(), lam=lam.cpu().numpy(),
                flags=flags.cpu().numpy(), kappa=kappa.cpu().numpy(), counters=cnt.cpu().numpy())


@pytest.mark.parametrize("name", list(CASES))
def test_amplitude_stats(gpu_lib, name):
    c = case(name)
    g = gpu_path(gpu_lib, c)
    np.testing.assert_allclose(g["mean"], c.orc["mean"], rtol=1e-13, atol=0)
    np.testing.assert_allclose(g["var"], c.orc["var"], rtol=1e-10, atol=1e-15 * np.max(c.orc["mean"]) ** 2)


@pytest.mark.parametrize("name", list(CASES))
def test_shp_masks_bit_exact(gpu_lib, name):
    c = case(name)
    g = gpu_path(gpu_lib, c)
    wl = c.wl
    band = np.abs(c.stat - O.glrt_threshold(wl.alpha)) < O.GLRT_BAND  # [oR, oC, W]
    bg = O.mask_bits(g["mask"], wl.window)
    bo = O.mask_bits(c.orc["mask"], wl.window)
    diff = (bg != bo) & ~band
    print(f"[parity] {name}: band cases {int(band.sum())}, gpu band count {int(g['counters'][0])}")
    assert not diff.any(), f"{int(diff.sum())} mask bits differ outside the band"
    np.testing.assert_array_equal(g["count"][~band.any(-1)], c.orc["count"][~band.any(-1)])
    # padding bits above W stay clear
    W = bo.shape[-1]
    if W % 32:
        assert np.all(g["mask"][..., -1] >> np.uint32(W % 32) == 0)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("name", list(CASES))
def test_coherence(gpu_lib, name, prec):
    c = case(name)
    g = gpu_path(gpu_lib, c, prec)
    # same masks (previous test), so the matrices are comparable pixel by pixel
    ok = np.all(np.isfinite(c.orc["coh"].reshape(len(c.sens), -1)), axis=1)
    _, dmax = coherence_error(g["coh"], c.orc["coh"])
    d = np.abs(g["coh"][ok].astype(np.complex128) - c.orc["coh"][ok])
    print(f"[parity] {name} {prec}: max |dC| {dmax:.3e}, mean {d.mean():.3e} (bound {EPS[prec]:.1e})")
    assert dmax <= COH_TOL
    assert dmax <= EPS[prec]  # the bound the phase criterion assumes
    # Hermitian with an exact unit diagonal
    gc = g["coh"][ok]
    assert np.all(gc[:, np.arange(c.wl.N), np.arange(c.wl.N)] == 1)
    np.testing.assert_allclose(gc, np.conj(np.swapaxes(gc, 1, 2)), atol=2e-6)
    assert np.all(np.isnan(g["coh"][~ok]))


@pytest.mark.parametrize("name", list(CASES))
def test_phase_link_on_oracle_coherence(gpu_lib, name):
    """The eigen-solver alone, fed the oracle's matrices rounded to complex64."""
    c = case(name)
    C64 = torch.from_numpy(c.orc["coh"].astype(np.complex64)).cuda()
    cnt = gpu_lib.new_counters()
    ph, lam, flags = gpu_lib.phase_link(C64, ref=c.ref, counters=cnt)
    ph, lam, flags = ph.cpu().numpy(), lam.cpu().numpy(), flags.cpu().numpy()
    link = c.orc["link"]
    dC, _ = coherence_error(c.orc["coh"].astype(np.complex64), c.orc["coh"])
    err = phase_errors(ph, link["phasor"])
    # the input is C rounded to complex64: eps = the largest rounding, 1e-7
    out = check_phases(f"{name} linking only", err, c.sens, flags, link, "fp32", c.orc["coh"], dC_pix=dC,
                       min_well_posed=len(c.sens) // 10, eps=1e-7)
    print(f"[parity] {name}: counters {cnt.cpu().numpy()[:7]}")
    assert np.all(ph[c.ref] == 1)
    # eigenvalue of the returned vector on well-posed EMI pixels
    emi = (flags == 0) & (link["flag"] == 0) & (3 * c.sens * EPS["fp32"] <= PHASE_TOL)
    np.testing.assert_allclose(lam[emi], link["lam"][emi], rtol=1e-3)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("name", list(CASES))
def test_end_to_end_phases(gpu_lib, name, prec):
    c = case(name)
    g = gpu_path(gpu_lib, c, prec)
    link = c.orc["link"]
    dC, _ = coherence_error(g["coh"], c.orc["coh"])
    err = phase_errors(g["ph"], link["phasor"])
    check_phases(f"{name} end to end", err, c.sens, g["flags"], link, prec, c.orc["coh"], dC_pix=dC,
                 min_well_posed=len(c.sens) // 10)
    assert np.all(g["ph"][:, g["flags"] == O.FLAG_INVALID] == 1)


# every linking-kernel variant (columns per row NJ = 12, 16, 20, 24, 28, 32; one
# or two rows per lane) and both coherence tiles (16 and 32 images), with the
# N = 15 + k stacks of the sequential scheme above 15 images
VARIANT_N = [3, 8, 12, 13, 16, 17, 20, 21, 22, 24, 25, 28, 29, 32]


@pytest.mark.parametrize("N", VARIANT_N)
def test_linking_variants_against_oracle(gpu_lib, N):
    n_new = min(N, 15)
    wl = synth.Workload(f"variant{N}", 99, 198, n_new, N - n_new, (11, 5, 6, 3), model="burst")
    z = synth.make_stack(wl, seed=300 + N)
    ref = max(0, wl.n_comp - 1)
    orc = O.link_ministack(z.numpy(), wl.n_comp, wl.window, wl.alpha, ref)
    sens = sensitivity(orc["coh"], ref)
    zc = z.cuda()
    mean, var = gpu_lib.amplitude_stats(zc[wl.n_comp:].contiguous())
    mask, _ = gpu_lib.shp_select(mean, var, wl.n_new, wl.window, wl.alpha)
    _, _, _, stat = O.shp_select(orc["mean"], orc["var"], wl.n_new, wl.window, wl.alpha, return_stat=True)
    band = np.abs(stat - O.glrt_threshold(wl.alpha)) < O.GLRT_BAND
    diff = (O.mask_bits(mask.cpu().numpy().view(np.uint32), wl.window) != O.mask_bits(orc["mask"], wl.window))
    assert not (diff & ~band).any()
    for prec in ("fp32", "bf16"):
        coh = gpu_lib.estimate_coherence(zc, mask, wl.window, precision=prec)
        ph, lam, flags = gpu_lib.phase_link(coh, ref=ref)
        dC, dmax = coherence_error(coh.cpu().numpy(), orc["coh"])
        assert dmax <= min(COH_TOL, EPS[prec]), f"N={N} {prec}: max |dC| {dmax:.2e}"
        err = phase_errors(ph.cpu().numpy(), orc["link"]["phasor"])
        check_phases(f"N={N} (99x198)", err, sens, flags.cpu().numpy(), orc["link"], prec, orc["coh"], dC_pix=dC,
                     min_well_posed=len(sens) // 10)


@pytest.mark.parametrize("name", list(CASES))
def test_compress_on_oracle_phasors(gpu_lib, name):
    c = case(name)
    wl = c.wl
    oR, oC = wl.out_shape
    ph = torch.from_numpy(c.orc["phasor"].astype(np.complex64)).cuda().contiguous()
    k = gpu_lib.compress_ministack(c.stack.cuda(), c.first_real, wl.window, ph).cpu().numpy()
    want = O.compress(c.z, c.first_real, c.orc["phasor"].astype(np.complex64), wl.window)
    scale = np.abs(c.z[c.first_real:]).astype(np.float64).sum(0)
    assert np.max(np.abs(k - want) / scale) <= 1e-6


def test_merge_amplitude_stats(gpu_lib):
    rng = np.random.default_rng(21)
    G, R, C = 5, 37, 53
    means = rng.uniform(0.1, 3, (G, R, C))
    var = rng.uniform(0.0, 2, (G, R, C))
    w = [15, 15, 15, 7, 3]
    mo, vo = O.merge_amplitude_stats(list(means), list(var), w)
    mg, vg = gpu_lib.merge_amplitude_stats(torch.from_numpy(means).cuda(), torch.from_numpy(var).cuda(), w)
    np.testing.assert_allclose(mg.cpu().numpy(), mo, rtol=1e-14)
    np.testing.assert_allclose(vg.cpu().numpy(), vo, rtol=1e-11, atol=1e-14)


# ------------------------------------------------------------------ edge cases
def test_two_images_closed_form(gpu_lib):
    rng = np.random.default_rng(22)
    P = 1000
    g = rng.uniform(0.05, 0.99, P)
    th = rng.uniform(-np.pi, np.pi, P)
    Cm = np.zeros((P, 2, 2), np.complex64)
    Cm[:, 0, 0] = Cm[:, 1, 1] = 1
    Cm[:, 1, 0] = g * np.exp(1j * th)
    Cm[:, 0, 1] = g * np.exp(-1j * th)
    ph, lam, flags = gpu_lib.phase_link(torch.from_numpy(Cm).cuda(), ref=0)
    ph = ph.cpu().numpy()
    assert np.all(flags.cpu().numpy() == 0)
    assert np.abs(np.angle(ph[1] * np.exp(-1j * th))).max() < 1e-5
    np.testing.assert_allclose(lam.cpu().numpy(), 1.0, atol=1e-4)


def test_upper_triangle_reading_above_16_images(gpu_lib):
    """For N > 16 the linking kernel takes C as the Hermitian matrix of its
    upper triangle (two rows per lane keep B as a packed triangle): changing
    the strictly lower triangle by a few ulp leaves every output bit
    unchanged, including on ill-conditioned |C|, where the inverses of the
    two triangles of |C| differ most.  On well-posed pixels the phases match
    the FP64 oracle on that Hermitian matrix."""
    rng = np.random.default_rng(31)
    N, P, ref = 25, 512, 3
    looks = rng.integers(N + 2, 3 * N, P)
    Ch = np.empty((P, N, N), np.complex128)
    for p in range(P):
        Z = rng.standard_normal((N, looks[p])) + 1j * rng.standard_normal((N, looks[p]))
        # correlated images; the stronger the common part, the closer |C| gets to singular
        Z[1:] += [2.0, 6.0, 15.0][p % 3] * Z[:1] * np.exp(1j * rng.uniform(-np.pi, np.pi, (N - 1, 1)))
        A = Z @ Z.conj().T
        d = 1.0 / np.sqrt(np.real(np.diag(A)))
        Ch[p] = A * d[:, None] * d[None, :]
    Ch = np.triu(Ch, 1) + np.conj(np.swapaxes(np.triu(Ch, 1), 1, 2)) + np.eye(N)
    Ch = Ch.astype(np.complex64)  # exactly Hermitian in FP32, unit diagonal
    assert np.array_equal(Ch, np.conj(np.swapaxes(Ch, 1, 2)))
    Cp = Ch.copy()
    low = np.tril(np.ones((N, N), bool), -1)
    ulp = np.float32(2.0 ** -22)
    Cp[:, low] = (Ch[:, low].real * (1 + ulp * rng.choice([-1, 1], (P, low.sum())))
                  + 1j * Ch[:, low].imag * (1 + ulp * rng.choice([-1, 1], (P, low.sum())))).astype(np.complex64)
    assert not np.array_equal(Cp, Ch)
    out = [gpu_lib.phase_link(torch.from_numpy(c).cuda(), ref=ref) for c in (Ch, Cp)]
    torch.cuda.synchronize()
    for a, b in zip(out[0], out[1]):
        assert torch.equal(a, b)
    cond = np.linalg.cond(np.abs(Ch.astype(np.complex128)))
    orc = O.phase_link(Ch, ref=ref)
    ph, lam, flags = (t.cpu().numpy() for t in out[0])
    sens = sensitivity(Ch.astype(np.complex128), ref)
    print(f"[parity] upper triangle N={N}: max cond(|C|) {cond.max():.1e}", flush=True)
    # the input is exactly Hermitian in FP32: only the solver's rounding remains
    check_phases("upper triangle N=25", phase_errors(ph, orc["phasor"]), sens, flags, orc, "fp32",
                 Ch.astype(np.complex128), min_well_posed=P // 10, eps=1e-7)


def test_nodata_pixels_are_invalid_and_ragged_grid(gpu_lib):
    wl = synth.crop("tiny", 37, 43)
    z = synth.make_stack(wl, seed=23)
    z[:, 5:9, 7:12] = 0  # nodata block
    window = (3, 2, 2, 3)  # ragged: 37 = 12*3 + 1, 43 = 21*2 + 1
    zc = z.cuda()
    mean, var = gpu_lib.amplitude_stats(zc)
    mask, count = gpu_lib.shp_select(mean, var, wl.n_new, window, 1e-3)
    coh = gpu_lib.estimate_coherence(zc, mask, window)
    ph, lam, flags = gpu_lib.phase_link(coh, ref=0)
    r = O.link_ministack(z.numpy(), 0, window, 1e-3, 0)
    np.testing.assert_array_equal(mask.cpu().numpy().view(np.uint32), r["mask"])
    np.testing.assert_array_equal(flags.cpu().numpy() == 2, r["link"]["flag"] == 2)
    assert (r["link"]["flag"] == 2).sum() > 0
    inval = flags.cpu().numpy() == 2
    assert np.all(ph.cpu().numpy()[:, inval] == 1)


def test_nan_nodata_outside_shps_is_excluded(gpu_lib):
    """A NaN nodata block: never an SHP of another pixel (Sec. 3.1, nodata
    reading), so the pixels whose windows reach it have the oracle's finite
    coherence in both precisions, also where a NaN pixel and an SHP share a
    pixel-pair record; only the pixels centred on the block are invalid."""
    wl = synth.crop("tiny", 37, 43)
    z = synth.make_stack(wl, seed=26)
    z[:, 5:9, 7:12] = complex(float("nan"), float("nan"))
    window = (3, 2, 2, 3)
    zc = z.cuda()
    mean, var = gpu_lib.amplitude_stats(zc)
    mask, count = gpu_lib.shp_select(mean, var, wl.n_new, window, 1e-3)
    r = O.link_ministack(z.numpy(), 0, window, 1e-3, 0)
    np.testing.assert_array_equal(mask.cpu().numpy().view(np.uint32), r["mask"])
    P = len(r["coh"])
    fin = np.all(np.isfinite(r["coh"].reshape(P, -1)), axis=1)
    assert fin.sum() > 0 and (~fin).sum() > 0
    for prec in ("fp32", "bf16"):
        coh = gpu_lib.estimate_coherence(zc, mask, window, precision=prec)
        ph, lam, flags = gpu_lib.phase_link(coh, ref=0)
        g = coh.cpu().numpy().reshape(P, -1)
        assert np.all(np.isfinite(g[fin])), prec
        assert np.all(np.isnan(g[~fin])), prec
        assert np.max(np.abs(g[fin] - r["coh"].reshape(P, -1)[fin])) < COH_TOL, prec
        np.testing.assert_array_equal(flags.cpu().numpy() == 2, r["link"]["flag"] == 2)


def test_max_images_and_single_image(gpu_lib):
    wl = synth.crop("tiny", 24, 24)
    rng = np.random.default_rng(24)
    for N in (1, 32):
        z = (rng.normal(size=(N, 24, 24)) + 1j * rng.normal(size=(N, 24, 24))).astype(np.complex64)
        z += 2 * z[:1]
        window = (2, 2, 2, 2)
        zc = torch.from_numpy(z).cuda()
        mean, var = gpu_lib.amplitude_stats(zc)
        mask, _ = gpu_lib.shp_select(mean, var, N, window, 1e-3)
        coh = gpu_lib.estimate_coherence(zc, mask, window, precision="bf16")
        ph, lam, flags = gpu_lib.phase_link(coh, ref=N - 1)
        r = O.link_ministack(z, 0, window, 1e-3, N - 1)
        np.testing.assert_array_equal(mask.cpu().numpy().view(np.uint32), r["mask"])
        d = np.abs(coh.cpu().numpy() - r["coh"])
        assert np.nanmax(d) < COH_TOL
        if N == 1:
            assert np.all(ph.cpu().numpy() == 1)


def test_window_larger_than_image(gpu_lib):
    wl = synth.crop("tiny", 7, 9)
    z = synth.make_stack(wl, seed=25)
    window = (11, 5, 1, 1)
    zc = z.cuda()
    mean, var = gpu_lib.amplitude_stats(zc)
    mask, count = gpu_lib.shp_select(mean, var, wl.n_new, window, 1e-3)
    coh = gpu_lib.estimate_coherence(zc, mask, window)
    r = O.link_ministack(z.numpy(), 0, window, 1e-3, 0)
    np.testing.assert_array_equal(mask.cpu().numpy().view(np.uint32), r["mask"])
    assert np.nanmax(np.abs(coh.cpu().numpy() - r["coh"])) < COH_TOL


def test_empty_pixel_list(gpu_lib):
    coh = torch.zeros((0, 5, 5), dtype=torch.complex64, device="cuda")
    ph, lam, flags = gpu_lib.phase_link(coh)
    assert ph.shape == (5, 0)


def test_deterministic(gpu_lib):
    c = case("burst-crop")
    a = gpu_path(gpu_lib, c, "bf16")
    b = gpu_path(gpu_lib, c, "bf16")
    for k in ("mask", "coh", "ph", "kappa"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k
