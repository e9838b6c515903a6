"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign, index or conjugation, a transposed operand, an off-by-one in the
window) fails at least one of them.  None of them re-types the oracle's own
formula and compares it with itself.
"""
import math
import os

import numpy as np
import pytest
from scipy import special

from oracle import plink_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- geometry
def test_window_table_matches_paper_convention():
    """Supplement table: full window = 2h+1, half-window written (x, y)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "shp_windows.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 5
    for name, hx, hy, X, Y in rows:
        hx, hy, X, Y = map(int, (hx, hy, X, Y))
        offs = O.window_offsets((hx, hy, 6, 3))
        dxs = sorted({dx for _, dx in offs})
        dys = sorted({dy for dy, _ in offs})
        assert len(dxs) == X and len(dys) == Y, name
        assert len(offs) == X * Y
        assert O.mask_words((hx, hy, 6, 3)) == (X * Y + 31) // 32


def test_output_grid_centres_inside_and_stride():
    R, C, w = 2048, 8192, (11, 5, 6, 3)
    oR, oC = O.output_grid(R, C, w)
    assert (oR, oC) == (682, 1365)
    cy, cx = O.output_centres(R, C, w)
    assert cy[0] == 1 and cx[0] == 3 and cy[-1] < R and cx[-1] < C
    assert np.all(np.diff(cy) == 3) and np.all(np.diff(cx) == 6)


# ---------------------------------------------------------------- statistics
def test_amplitude_stats_closed_forms():
    rng = np.random.default_rng(1)
    ph = np.exp(1j * rng.uniform(-np.pi, np.pi, (8, 3, 4)))
    amp = np.array([2.0, 4.0] * 4)[:, None, None] * np.ones((8, 3, 4))
    mean, var = O.amplitude_stats(amp * ph)
    np.testing.assert_allclose(mean, 3.0, rtol=1e-14)
    np.testing.assert_allclose(var, 1.0, rtol=1e-13)  # ((4-2)/2)^2, population
    mean, var = O.amplitude_stats(np.full((5, 2, 2), 3 - 4j, np.complex64))
    np.testing.assert_allclose(mean, 5.0)
    np.testing.assert_allclose(var, 0.0, atol=1e-14)


def test_merge_equals_stats_of_concatenation():
    rng = np.random.default_rng(2)
    groups = [rng.normal(size=(m, 5, 6)) + 1j * rng.normal(size=(m, 5, 6)) for m in (15, 15, 7, 1)]
    st = [O.amplitude_stats(g) for g in groups]
    mu, var = O.merge_amplitude_stats([s[0] for s in st], [s[1] for s in st],
                                      [g.shape[0] for g in groups])
    mu_d, var_d = O.amplitude_stats(np.concatenate(groups))
    np.testing.assert_allclose(mu, mu_d, rtol=1e-13)
    np.testing.assert_allclose(var, var_d, rtol=1e-11, atol=1e-13)


# ---------------------------------------------------------------- GLRT
def test_chi2_threshold_is_squared_normal_quantile():
    for alpha in (1e-3, 1e-2, 0.05):
        thr = O.glrt_threshold(alpha)
        z = special.ndtri(1 - alpha / 2)
        assert abs(thr - z * z) < 1e-9 * thr
        assert abs(math.erfc(math.sqrt(thr / 2)) - alpha) < 1e-12
    assert abs(O.glrt_threshold(1e-3) - 10.827566170662733) < 1e-9


def test_glrt_statistic_closed_form_and_invariants():
    n = 15
    for r in (1.0, 2.0, 3.7, 100.0):
        t = O.glrt_statistic(1.0, r, n)
        assert abs(t - 2 * n * math.log((1 + r) ** 2 / (4 * r))) < 1e-12 * max(1, t)
        assert abs(O.glrt_statistic(r, 1.0, n) - t) < 1e-12 * max(1, t)   # symmetric
        assert abs(O.glrt_statistic(5 * r, 5.0, n) - t) < 1e-11 * max(1, t)  # scale-free
    assert O.glrt_statistic(2.5, 2.5, n) == 0.0
    # a persistent scatterer at 10x amplitude against a distributed scatterer:
    # scale ratio 100 -> T = 2n ln 25.5025 > threshold for every n >= 2
    thr = O.glrt_threshold(1e-3)
    for n in range(2, 40):
        assert O.glrt_statistic(100.0, 1.0, n) > thr


def test_glrt_false_alarm_rate_iid_rayleigh():
    """Under H0 (same scale), rejections happen at rate ~alpha."""
    rng = np.random.default_rng(3)
    n, pairs, alpha = 15, 200_000, 1e-2
    z = (rng.normal(size=(2, n, pairs)) + 1j * rng.normal(size=(2, n, pairs))) / np.sqrt(2)
    m0, v0 = O.amplitude_stats(z[0][:, None, :])
    m1, v1 = O.amplitude_stats(z[1][:, None, :])
    t = O.glrt_statistic(O.rayleigh_scale(m0, v0), O.rayleigh_scale(m1, v1), n)
    rate = float(np.mean(t > O.glrt_threshold(alpha)))
    assert 0.8 * alpha < rate < 1.3 * alpha, rate


def _brute_mask(mean, var, n, window, alpha):
    R, C = mean.shape
    hx, hy, sx, sy = window
    thr = O.glrt_threshold(alpha)
    oR, oC = R // sy, C // sx
    W = (2 * hx + 1) * (2 * hy + 1)
    nw = (W + 31) // 32
    mask = np.zeros((oR, oC, nw), np.uint32)
    for oy in range(oR):
        for ox in range(oC):
            py, px = oy * sy + sy // 2, ox * sx + sx // 2
            sp = (mean[py, px] ** 2 + var[py, px]) / 2
            b = 0
            for dy in range(-hy, hy + 1):
                for dx in range(-hx, hx + 1):
                    qy, qx = py + dy, px + dx
                    ok = False
                    if dy == 0 and dx == 0:
                        ok = True
                    elif 0 <= qy < R and 0 <= qx < C and sp > 0:
                        sq = (mean[qy, qx] ** 2 + var[qy, qx]) / 2
                        if sq > 0:
                            t = 2 * n * (2 * math.log((sp + sq) / 2) - math.log(sp) - math.log(sq))
                            ok = t <= thr
                    if ok:
                        mask[oy, ox, b // 32] |= np.uint32(1 << (b % 32))
                    b += 1
    return mask


@pytest.mark.parametrize("window", [(2, 1, 1, 1), (3, 2, 3, 2), (1, 3, 2, 3)])
def test_shp_mask_bruteforce(window):
    rng = np.random.default_rng(4)
    R, C = 9, 11
    mean = np.exp(rng.normal(0, 0.6, (R, C)))
    var = mean ** 2 * rng.uniform(0.1, 0.5, (R, C))
    mean[4, 5] = 0.0
    var[4, 5] = 0.0  # nodata pixel: never an SHP, its own mask holds itself only
    mask, count, band = O.shp_select(mean, var, 12, window, 0.05)
    ref = _brute_mask(mean, var, 12, window, 0.05)
    np.testing.assert_array_equal(mask, ref)
    bits = O.mask_bits(mask, window)
    np.testing.assert_array_equal(count, bits.sum(-1))
    assert count.min() >= 1


# ---------------------------------------------------------------- coherence
def _exp_gamma(N, g0=0.8, ginf=0.1, tau=5.0):
    t = np.arange(N)
    G = (g0 - ginf) * np.exp(-np.abs(t[:, None] - t[None, :]) / tau) + ginf
    np.fill_diagonal(G, 1.0)
    return G


def _full_mask(R, C, window):
    oR, oC = O.output_grid(R, C, window)
    W = (2 * window[0] + 1) * (2 * window[1] + 1)
    m = np.zeros((oR, oC, (W + 31) // 32), np.uint32)
    for b in range(W):
        m[..., b // 32] |= np.uint32(1 << (b % 32))
    return m


def test_coherence_invariants_random():
    rng = np.random.default_rng(5)
    N, R, C, w = 6, 10, 12, (2, 2, 1, 1)
    z = (rng.normal(size=(N, R, C)) + 1j * rng.normal(size=(N, R, C))).astype(np.complex64)
    Cm, valid = O.coherence(z, _full_mask(R, C, w), w)
    assert valid.all()
    np.testing.assert_allclose(Cm, np.conj(np.swapaxes(Cm, 1, 2)), atol=1e-15)
    np.testing.assert_allclose(np.einsum("pii->pi", Cm), 1.0, atol=1e-14)
    assert np.abs(Cm).max() <= 1 + 1e-12
    assert np.linalg.eigvalsh(Cm).min() > -1e-12
    # per-image scaling invariance: |C| unchanged, phases move by the scale's phase
    s = (rng.uniform(0.5, 2, N) * np.exp(1j * rng.uniform(-3, 3, N)))
    C2, _ = O.coherence(z * s[:, None, None].astype(np.complex64), _full_mask(R, C, w), w)
    u = s / np.abs(s)
    np.testing.assert_allclose(C2, Cm * u[None, :, None] * np.conj(u)[None, None, :], atol=1e-6)


def test_coherence_single_sample_is_rank_one_phasor():
    rng = np.random.default_rng(6)
    N, R, C, w = 5, 7, 7, (1, 1, 1, 1)
    z = (rng.normal(size=(N, R, C)) + 1j * rng.normal(size=(N, R, C))).astype(np.complex64)
    mask = np.zeros((R, C, 1), np.uint32)
    mask[..., 0] = 1 << 4  # centre bit only
    Cm, _ = O.coherence(z, mask, w)
    u = z.astype(np.complex128).reshape(N, -1).T
    u = u / np.abs(u)
    np.testing.assert_allclose(Cm, u[:, :, None] * np.conj(u[:, None, :]), atol=1e-12)


def test_coherence_orthogonal_samples_reproduce_model():
    """z^(l) = sqrt(N) Phi Gamma^(1/2) e_l for l = 1..N sums to N Phi Gamma Phi^H."""
    N = 5
    G = _exp_gamma(N)
    w_, V = np.linalg.eigh(G)
    Gh = V @ np.diag(np.sqrt(w_)) @ V.T
    phi = np.array([0.0, 0.7, -1.2, 2.9, -2.5])
    samples = np.sqrt(N) * (np.exp(1j * phi)[:, None] * Gh)  # column l = sample l
    # lay the N samples on a 1 x N image; one output pixel whose window is the row
    z = samples[:, None, :].astype(np.complex128)
    w = (2, 0, 5, 1)  # half_x 2, stride_x 5 -> output (0, 0) centred at x = 2
    Cm, valid = O.coherence(z, _full_mask(1, N, w), w)
    np.testing.assert_allclose(Cm[0], np.exp(1j * phi)[:, None] * G * np.exp(-1j * phi)[None, :],
                               atol=1e-13)


def test_coherence_bruteforce_two_pixels():
    rng = np.random.default_rng(7)
    N, R, C, w = 4, 9, 13, (3, 2, 3, 2)
    z = rng.normal(size=(N, R, C)) + 1j * rng.normal(size=(N, R, C))
    mean, var = O.amplitude_stats(z)
    mask, count, _ = O.shp_select(mean, var, N, w, 0.2)
    Cm, _ = O.coherence(z, mask, w)
    oR, oC = O.output_grid(R, C, w)
    for oy, ox in [(0, 0), (oR - 1, oC - 1), (2, 1)]:
        py, px = oy * 2 + 1, ox * 3 + 1
        A = np.zeros((N, N), complex)
        b = 0
        for dy in range(-2, 3):
            for dx in range(-3, 4):
                if (int(mask[oy, ox, b // 32]) >> (b % 32)) & 1:
                    v = z[:, py + dy, px + dx]
                    A += np.outer(v, np.conj(v))
                b += 1
        d = np.sqrt(np.real(np.diag(A)))
        np.testing.assert_allclose(Cm[oy * oC + ox], A / np.outer(d, d), atol=1e-13)


# ---------------------------------------------------------------- phase linking
def test_noise_free_model_recovers_true_phase_emi_and_evd():
    N, ref = 15, 3
    rng = np.random.default_rng(8)
    phi = rng.uniform(-np.pi, np.pi, N)
    Cm = (np.exp(1j * phi)[:, None] * _exp_gamma(N) * np.exp(-1j * phi)[None, :])[None]
    for method in ("emi", "evd"):
        out = O.phase_link(Cm, ref=ref, method=method)
        err = O.wrap(out["phase"][:, 0] - (phi - phi[ref]))
        assert np.abs(err).max() < 1e-10, method
        assert out["phasor"][ref, 0] == 1.0
    out = O.phase_link(Cm, ref=ref)
    assert out["flag"][0] == O.FLAG_EMI
    assert abs(out["lam"][0] - 1.0) < 1e-10  # lambda_min(Gamma^-1 o Gamma) = 1


def test_two_image_closed_form():
    for g, th in [(0.3, 1.1), (0.95, -2.0), (0.5, 3.0)]:
        Cm = np.array([[[1, g * np.exp(-1j * th)], [g * np.exp(1j * th), 1]]])
        out = O.phase_link(Cm, ref=0)
        assert abs(O.wrap(out["phase"][1, 0] - th)) < 1e-12
        assert abs(out["lam"][0] - 1.0) < 1e-12
        np.testing.assert_allclose(O.ldl_pivots(np.abs(Cm))[0], [1.0, 1.0 - g * g], rtol=1e-14)


def _eig3_closed_form(H):
    """Eigenvalues of a 3x3 Hermitian matrix by the trigonometric cubic formula
    and the smallest one's eigenvector from a cross product of two rows."""
    a = np.trace(H).real / 3
    B = H - a * np.eye(3)
    p = math.sqrt(np.real(np.trace(B @ B)) / 6)
    r = np.real(np.linalg.det(B / p)) / 2
    r = min(1.0, max(-1.0, r))
    ph = math.acos(r) / 3
    lam = sorted(a + 2 * p * math.cos(ph + 2 * math.pi * k / 3) for k in range(3))
    M = H - lam[0] * np.eye(3)
    v = np.cross(M[0], M[1])  # bilinear: M[0] . v = M[1] . v = 0
    return lam, v / np.linalg.norm(v)


def test_three_image_against_closed_form_eigen():
    rng = np.random.default_rng(9)
    for _ in range(5):
        z = rng.normal(size=(3, 40)) + 1j * rng.normal(size=(3, 40))
        z[1] += 0.8 * z[0]
        z[2] += 0.5 * z[1]
        A = z @ z.conj().T
        d = np.sqrt(np.real(np.diag(A)))
        Cm = A / np.outer(d, d)
        H = np.linalg.inv(np.abs(Cm)) * Cm
        lam, v = _eig3_closed_form(H)
        out = O.phase_link(Cm[None], ref=0)
        want = np.angle(v * np.conj(v[0]))
        assert abs(out["lam"][0] - lam[0]) < 1e-9
        assert np.abs(O.wrap(out["phase"][:, 0] - want)).max() < 1e-9


def test_phase_screen_shifts_linked_phase_exactly():
    """z_i -> z_i exp(j d_i) moves every linked phase by d_i - d_ref."""
    rng = np.random.default_rng(10)
    N, R, C, w, ref = 7, 12, 12, (2, 2, 3, 3), 2
    z = rng.normal(size=(N, R, C)) + 1j * rng.normal(size=(N, R, C))
    z += 1.5 * (rng.normal(size=(1, R, C)) + 1j * rng.normal(size=(1, R, C)))
    d = rng.uniform(-np.pi, np.pi, N)
    r0 = O.link_ministack(z, 0, w, 1e-3, ref)
    r1 = O.link_ministack(z * np.exp(1j * d)[:, None, None], 0, w, 1e-3, ref)
    np.testing.assert_array_equal(r0["mask"], r1["mask"])
    diff = O.wrap(r1["link"]["phase"] - r0["link"]["phase"] - (d - d[ref])[:, None])
    assert np.abs(diff).max() < 1e-9


def _random_abs_coherence(rng, N, looks):
    z = rng.normal(size=(N, looks)) + 1j * rng.normal(size=(N, looks))
    z[1:] += rng.uniform(0.2, 1.5) * z[:1]
    A = z @ z.conj().T
    d = np.sqrt(np.real(np.diag(A)))
    return np.abs(A / np.outer(d, d))


@pytest.mark.parametrize("N", [3, 4, 7, 12, 16, 20, 25, 32])
def test_ldl_pivots_are_squared_cholesky_diagonal(N):
    """The unpivoted LDL^T pivots of an SPD matrix are the squares of its
    Cholesky diagonal (LAPACK) and the ratios of consecutive leading principal
    minors; their product is det G."""
    rng = np.random.default_rng(100 + N)
    G = np.stack([_random_abs_coherence(rng, N, 3 * N + k) for k in range(6)])
    d = O.ldl_pivots(G)
    L = np.linalg.cholesky(G)
    np.testing.assert_allclose(d, np.einsum("pii->pi", L) ** 2, rtol=1e-10)
    for p in range(len(G)):
        minors = np.array([np.linalg.det(G[p, :k, :k]) for k in range(1, N + 1)])
        np.testing.assert_allclose(d[p], minors / np.concatenate([[1.0], minors[:-1]]), rtol=1e-8)
        np.testing.assert_allclose(np.prod(d[p]), np.linalg.det(G[p]), rtol=1e-8)


def _unit_diag_from_ldl(Lstrict, d0_target, k):
    """A unit-diagonal SPD matrix G = L D L^T with nonnegative entries whose
    LDL^T pivot number k is d0_target: every pivot is 1 - sum_j L_ij^2 d_j."""
    N = Lstrict.shape[0]
    L = np.eye(N) + np.tril(Lstrict, -1)
    d = np.zeros(N)
    for i in range(N):
        if i == k:
            # rescale row k's multipliers so that its pivot is the target
            s = np.sum(L[i, :i] ** 2 * d[:i])
            L[i, :i] *= np.sqrt((1.0 - d0_target) / s)
        d[i] = 1.0 - np.sum(L[i, :i] ** 2 * d[:i])
        assert d[i] > 0
    return L @ np.diag(d) @ L.T, d


@pytest.mark.parametrize("k", [2, 5, 9])
def test_fallback_decided_by_a_deep_pivot(k):
    """A pivot at index k >= 2 just below / above tau switches EMI to EVD;
    built from a prescribed LDL^T so that the pivot is known exactly."""
    rng = np.random.default_rng(200 + k)
    N = 12
    Ls = rng.uniform(0.0, 0.25, (N, N))
    phi = rng.uniform(-np.pi, np.pi, N)
    for target, want in ((0.5 * O.TAU_PIVOT, O.FLAG_EVD), (2.0 * O.TAU_PIVOT, O.FLAG_EMI)):
        G, d = _unit_diag_from_ldl(Ls, target, k)
        np.testing.assert_allclose(np.diag(G), 1.0, atol=1e-14)
        assert np.all(np.delete(d, k) > 1e-3)  # only pivot k is small
        np.testing.assert_allclose(O.ldl_pivots(G[None])[0], d, rtol=1e-7, atol=1e-12)
        Cm = np.exp(1j * phi)[:, None] * G * np.exp(-1j * phi)[None, :]
        out = O.phase_link(Cm[None], ref=0)
        assert out["flag"][0] == want, (k, target)
        assert abs(out["min_pivot"][0] - target) < 1e-3 * target
        # noise-free model: either branch recovers the phases exactly
        assert np.abs(O.wrap(out["phase"][:, 0] - (phi - phi[0]))).max() < 1e-6


def test_fallback_rule_rank_one_is_evd_and_exact():
    N = 6
    phi = np.linspace(-3, 3, N)
    Cm = np.exp(1j * (phi[:, None] - phi[None, :]))[None]
    out = O.phase_link(Cm, ref=0)
    assert out["flag"][0] == O.FLAG_EVD and out["min_pivot"][0] <= O.TAU_PIVOT
    assert np.abs(O.wrap(out["phase"][:, 0] - (phi - phi[0]))).max() < 1e-10
    assert abs(out["lam"][0] - N) < 1e-10


def test_invalid_pixel_flag_and_unit_phasors():
    Cm = np.full((1, 4, 4), np.nan + 0j)
    out = O.phase_link(Cm, ref=0)
    assert out["flag"][0] == O.FLAG_INVALID
    np.testing.assert_array_equal(out["phasor"][:, 0], 1.0)


# ---------------------------------------------------------------- compressed SLC
def test_compress_noise_free_reference_phase_factors_out():
    rng = np.random.default_rng(11)
    N, R, C, w, ref = 6, 7, 10, (1, 1, 3, 2), 0
    oR, oC = O.output_grid(R, C, w)
    phi = rng.uniform(-3, 3, N)
    a = rng.uniform(0.5, 2, (N, R, C))
    z = a * np.exp(1j * phi)[:, None, None]
    ph = np.broadcast_to(np.exp(1j * (phi - phi[ref]))[:, None, None], (N, oR, oC))
    k = O.compress(z, 0, ph, w)
    np.testing.assert_allclose(k, np.exp(1j * phi[ref]) * a.sum(0), rtol=1e-13)
    # first_real skips the leading planes
    k2 = O.compress(z, 2, ph, w)
    np.testing.assert_allclose(k2, np.exp(1j * phi[ref]) * a[2:].sum(0), rtol=1e-13)


def test_compress_block_mapping_and_bounds():
    rng = np.random.default_rng(12)
    N, R, C, w = 3, 10, 14, (2, 1, 4, 3)  # ragged: 10 = 3*3+1, 14 = 3*4+2
    oR, oC = O.output_grid(R, C, w)
    z = rng.normal(size=(N, R, C)) + 1j * rng.normal(size=(N, R, C))
    ph = np.exp(1j * rng.uniform(-3, 3, (N, oR, oC)))
    k = O.compress(z, 0, ph, w)
    for y, x in [(0, 0), (9, 13), (8, 11), (5, 7)]:
        by, bx = min(y // 3, oR - 1), min(x // 4, oC - 1)
        assert abs(k[y, x] - np.sum(np.conj(ph[:, by, bx]) * z[:, y, x])) < 1e-12
    assert np.all(np.abs(k) <= np.abs(z).sum(0) + 1e-12)
    z2 = rng.normal(size=z.shape) + 0j
    np.testing.assert_allclose(O.compress(z + z2, 0, ph, w), k + O.compress(z2, 0, ph, w),
                               atol=1e-12)


# ---------------------------------------------------------------- sequential
def _coherent_sequence(T, R, C, seed=13, noise=0.0):
    rng = np.random.default_rng(seed)
    # phases shared by every pixel of an epoch, so each window is coherent
    phi = np.broadcast_to(np.cumsum(rng.uniform(-1, 1, (T, 1, 1)), axis=0), (T, R, C))
    w = rng.normal(size=(R, C)) + 1j * rng.normal(size=(R, C))
    n = rng.normal(size=(T, R, C)) + 1j * rng.normal(size=(T, R, C))
    return np.exp(1j * phi) * (w[None] + noise * n), phi


def test_sequential_coherent_stack_referenced_to_day_one():
    M, K, R, C, w = 5, 2, 9, 9, (1, 1, 3, 3)
    z, phi = _coherent_sequence(4 * M, R, C)
    out = O.sequential([z[i * M:(i + 1) * M] for i in range(4)], K, w, 1e-3)
    cy, cx = O.output_centres(R, C, w)
    for k, o in enumerate(out):
        assert o["n_comp"] == min(k, K) and o["ref"] == (min(k, K) - 1 if k else 0)
        truth = phi[k * M:(k + 1) * M][:, cy][:, :, cx] - phi[0][cy][:, cx][None]
        err = O.wrap(np.angle(o["phasor"]) - truth)
        assert np.abs(err).max() < 1e-9, k
        # reference inheritance: every compressed SLC keeps the day-1 phase
        assert np.abs(O.wrap(np.angle(o["kappa"] * np.conj(out[0]["kappa"])))).max() < 1e-9


def test_sequential_is_append_only():
    M, K, R, C, w = 5, 2, 8, 8, (1, 1, 2, 2)
    z, _ = _coherent_sequence(3 * M, R, C, seed=14, noise=0.7)
    b = [z[i * M:(i + 1) * M] for i in range(3)]
    a2 = O.sequential(b[:2], K, w, 1e-3)
    a3 = O.sequential(b, K, w, 1e-3)
    for x, y in zip(a2, a3[:2]):
        np.testing.assert_array_equal(x["phasor"], y["phasor"])
        np.testing.assert_array_equal(x["kappa"], y["kappa"])


def test_sequential_statistics_window_and_n_eff():
    """Mini-stack k merges the amplitude statistics of mini-stacks k-K..k with
    n_eff = (K+1) M (reading R8).  Amplitudes are constant within each
    mini-stack, so the pooled Rayleigh scale of a pixel is half the mean of
    its squared amplitudes over the merged mini-stacks and every GLRT decision
    below follows from T = 2 n ln((s_p+s_q)^2 / (4 s_p s_q)) by hand:

      q1: amplitude 1.6 throughout: scale ratio 2.56, T = 0.4265 n: an SHP for
          n = 15 (6.4) and not for n >= 30 (12.8, 19.2)
      q2: amplitude 3 in mini-stack 0 only, then 1: at k = 3 (window 1..3)
          ratio 1 -> SHP; a window reaching back to 0 gives ratio 3 -> not
      q3: amplitude 2 in mini-stacks 1, 2, 1 in 3: window 1..3 ratio 3,
          T(45) = 25.9 -> not; the current mini-stack alone: ratio 1 -> SHP
      q4: amplitude 1 in 0..2, 3 in 3: window 1..3 ratio 11/3,
          T(45) = 35.6 -> not; mini-stacks 1..2 alone: ratio 1 -> SHP
    The centre pixel p has amplitude 1 throughout."""
    M, K, T = 15, 2, 4
    rng = np.random.default_rng(15)
    amp = np.ones((T, 3, 3))
    q1, q2, q3, q4 = (0, 0), (0, 2), (2, 0), (2, 2)  # window bits 0, 2, 6, 8
    amp[:, q1[0], q1[1]] = 1.6
    amp[0, q2[0], q2[1]] = 3.0
    amp[1:3, q3[0], q3[1]] = 2.0
    amp[3, q4[0], q4[1]] = 3.0
    batches = [amp[k][None] * np.exp(1j * rng.uniform(-np.pi, np.pi, (M, 3, 3))) for k in range(T)]
    out = O.sequential(batches, K, (1, 1, 3, 3), 1e-3)
    bits = [O.mask_bits(o["mask"], (1, 1, 3, 3))[0, 0] for o in out]
    # mini-stack 0: n = 15, window {0}
    assert bits[0][0] and not bits[0][2]  # q1 SHP at n = 15; q2: ratio 9 -> not
    # mini-stack 3: n = 45, window {1, 2, 3}
    assert not bits[3][0]
    assert bits[3][2]
    assert not bits[3][6]
    assert not bits[3][8]
    assert bits[3][4]  # the centre itself
    # the hand-computed statistics behind the decisions
    thr = O.glrt_threshold(1e-3)
    t = lambda r, n: 2 * n * math.log((1 + r) ** 2 / (4 * r))
    assert t(2.56, 15) < thr < t(2.56, 30)
    assert t(3.0, 45) > thr and t(11 / 3, 45) > thr and t(9.0, 15) > thr


# ---------------------------------------------------------------- adjoint
def _adjoint_case(seed, N=5, R=10, C=11, w=(2, 2, 3, 2)):
    rng = np.random.default_rng(seed)
    z = rng.normal(size=(N, R, C)) + 1j * rng.normal(size=(N, R, C))
    z += 1.2 * (rng.normal(size=(1, R, C)) + 1j * rng.normal(size=(1, R, C)))
    z *= np.exp(1j * rng.uniform(-3, 3, (N, 1, 1)))
    mean, var = O.amplitude_stats(z)
    mask, _, _ = O.shp_select(mean, var, N, w, 0.3)
    Cm, valid = O.coherence(z, mask, w)
    flags = O.phase_link(Cm, ref=1, valid=valid)["flag"]
    g = rng.normal(size=(N, len(flags)))
    return z, mask, w, flags, g


@pytest.mark.parametrize("method", ["emi", "evd"])
def test_adjoint_matches_central_finite_differences(method):
    z, mask, w, flags, g = _adjoint_case(41)
    if method == "evd":
        flags = np.where(flags == O.FLAG_INVALID, flags, O.FLAG_EVD).astype(np.uint8)
    assert np.any(flags == (O.FLAG_EMI if method == "emi" else O.FLAG_EVD))
    ref = 1
    grad = O.phase_link_vjp(z, mask, w, ref, g, flags)

    def loss(zz):
        ph = O.link_phases_fixed(zz, mask, w, ref, flags)
        return float(np.sum(g * ph))

    h = 1e-6
    rng = np.random.default_rng(42)
    N, R, C = z.shape
    idx = [(int(rng.integers(N)), int(rng.integers(R)), int(rng.integers(C))) for _ in range(40)]
    fd = np.zeros(len(idx), complex)
    for k, (i, y, x) in enumerate(idx):
        for part, unit in ((0, 1.0), (1, 1j)):
            zp, zm = z.copy(), z.copy()
            zp[i, y, x] += h * unit
            zm[i, y, x] -= h * unit
            dv = (loss(zp) - loss(zm)) / (2 * h)
            fd[k] += dv if part == 0 else 1j * dv
    an = np.array([grad[i, y, x] for (i, y, x) in idx])
    assert np.linalg.norm(an - fd) <= 1e-6 * np.linalg.norm(fd)


def test_adjoint_fd_at_the_differentiation_config():
    """The differentiation configuration's shape (N = 20, half-window 7 x 7,
    stride 1): the oracle's adjoint against FP64 central differences
    (h = 1e-6) at 64 random input pixels (a random image each, both real and
    imaginary parts), to 1e-6 relative."""
    import synth
    from adjoint_fd import fd_gradient
    wl = synth.crop("adjoint", 36, 36)
    z = synth.make_stack(wl, seed=51).numpy().astype(np.complex128)
    mean, var = O.amplitude_stats(z)
    mask, _, _ = O.shp_select(mean, var, wl.n_new, wl.window, wl.alpha)
    Cm, valid = O.coherence(z, mask, wl.window)
    ref = 2
    flags = O.phase_link(Cm, ref=ref, valid=valid)["flag"]
    rng = np.random.default_rng(52)
    g = rng.normal(size=(wl.N, len(flags)))
    grad = O.phase_link_vjp(z, mask, wl.window, ref, g, flags)
    entries = [(int(rng.integers(wl.N)), int(rng.integers(wl.R)), int(rng.integers(wl.C))) for _ in range(64)]
    fd = fd_gradient(z, mask, wl.window, ref, flags, g, entries)
    an = np.array([grad[n, y, x] for n, y, x in entries])
    assert np.linalg.norm(an - fd) <= 1e-6 * np.linalg.norm(fd)


def test_adjoint_phase_screen_closed_form():
    """z_i -> z_i exp(j d_i) moves phi_i by d_i - d_ref exactly, so the VJP
    contracted with dz = j d_i z_i equals sum_p sum_i g_i (d_i - d_ref)."""
    z, mask, w, flags, g = _adjoint_case(43)
    ref = 1
    grad = O.phase_link_vjp(z, mask, w, ref, g, flags)
    rng = np.random.default_rng(44)
    d = rng.normal(size=z.shape[0])
    dz = 1j * d[:, None, None] * z
    lhs = np.real(np.sum(np.conj(grad) * dz))
    ok = flags != O.FLAG_INVALID
    rhs = np.sum(g[:, ok] * (d - d[ref])[:, None])
    assert abs(lhs - rhs) <= 1e-9 * max(1.0, abs(rhs))
