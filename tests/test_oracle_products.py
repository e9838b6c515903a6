"""Pins of the FP64 oracle of the products built on the linked phases
(oracle/products.py) and of the driver options of the sequential scheme,
against statements of the paper, closed forms, hand-worked cases and library
solvers.  None re-types the oracle's own formula."""
import math

import numpy as np
import pytest
from scipy.optimize import linprog

from oracle import plink_oracle as O
from oracle import products as Q


# ---------------------------------------------------------------- temporal coherence
def test_temporal_coherence_two_images_is_one():
    """Sec. 3.3: with two images gamma_t is always 1 (EMI links them exactly)."""
    rng = np.random.default_rng(1)
    P = 200
    g = rng.uniform(0.05, 0.99, P)
    th = rng.uniform(-np.pi, np.pi, P)
    Cm = np.zeros((P, 2, 2), complex)
    Cm[:, 0, 0] = Cm[:, 1, 1] = 1
    Cm[:, 1, 0] = g * np.exp(1j * th)
    Cm[:, 0, 1] = np.conj(Cm[:, 1, 0])
    out = O.phase_link(Cm, ref=0)
    np.testing.assert_allclose(Q.temporal_coherence(Cm, out["phase"]), 1.0, atol=1e-12)


def test_temporal_coherence_noise_free_model_is_one():
    N = 12
    rng = np.random.default_rng(2)
    phi = rng.uniform(-np.pi, np.pi, N)
    t = np.arange(N)
    G = 0.7 * np.exp(-np.abs(t[:, None] - t[None, :]) / 5.0) + 0.1
    np.fill_diagonal(G, 1.0)
    Cm = (np.exp(1j * phi)[:, None] * G * np.exp(-1j * phi)[None, :])[None]
    out = O.phase_link(Cm, ref=4)
    assert abs(Q.temporal_coherence(Cm, out["phase"])[0] - 1.0) < 1e-12


def test_temporal_coherence_hand_example():
    """Interferogram phases 0 (0,1), pi/2 (0,2), pi (1,2) against zero linked
    phases: |1 + j - 1| / 3 = 1/3."""
    Cm = np.eye(3, dtype=complex)
    Cm[0, 1] = 0.5
    Cm[0, 2] = 0.5j
    Cm[1, 2] = -0.5
    Cm = Cm + np.triu(Cm, 1).conj().T
    assert abs(Q.temporal_coherence(Cm[None], np.zeros((3, 1)))[0] - 1.0 / 3.0) < 1e-15
    # the same with linked phases that undo two of the three: (0, 0, pi/2)
    # -> terms exp(j*0), exp(j(pi/2 - (0 - pi/2))) = -1, exp(j(pi - (0 - pi/2))) = -j
    g = Q.temporal_coherence(Cm[None], np.array([[0.0], [0.0], [np.pi / 2]]))[0]
    assert abs(g - abs(1 - 1 - 1j) / 3) < 1e-15


def test_temporal_coherence_bounds_and_phase_screen():
    rng = np.random.default_rng(3)
    N, R, C, w, ref = 8, 14, 16, (2, 2, 2, 2), 1
    z = rng.normal(size=(N, R, C)) + 1j * rng.normal(size=(N, R, C))
    z += 0.8 * (rng.normal(size=(1, R, C)) + 1j * rng.normal(size=(1, R, C)))
    r0 = O.link_ministack(z, 0, w, 1e-3, ref)
    g0 = Q.temporal_coherence(r0["coh"], r0["link"]["phase"], r0["link"]["flag"])
    assert np.all((g0 >= 0) & (g0 <= 1 + 1e-12)) and g0.min() < 0.99
    d = rng.uniform(-np.pi, np.pi, N)
    r1 = O.link_ministack(z * np.exp(1j * d)[:, None, None], 0, w, 1e-3, ref)
    g1 = Q.temporal_coherence(r1["coh"], r1["link"]["phase"], r1["link"]["flag"])
    np.testing.assert_allclose(g1, g0, atol=1e-10)


# ---------------------------------------------------------------- phase similarity
def test_network_size_is_three_m_minus_six():
    """Sec. 3.4: the nearest-3 network of M images has 3M - 6 interferograms."""
    for M in range(4, 33):
        net = Q.nearest_network(M, 3)
        assert len(net) == 3 * M - 6
        assert all(1 <= b - a <= 3 for a, b in net) and len(set(net)) == len(net)


def test_disk_offsets_gauss_circle_counts():
    # lattice points in a disk of radius r, minus the centre (OEIS A000328 - 1)
    for r, n in [(1, 4), (2, 12), (3, 28), (4, 48), (7, 148)]:
        assert len(Q.disk_offsets(r)) == n


def test_phase_similarity_hand_example():
    """1 x 3 grid, two images (one interferogram), radius 1: the centre's
    neighbours differ by 0.5 and 1.2 rad, so gamma_s is the mean of the two
    cosines (median of two values); each end has the centre as its only
    neighbour."""
    ph = np.zeros((2, 1, 3))
    ph[1, 0, 0] = 0.5
    ph[1, 0, 2] = 1.2
    g = Q.phase_similarity(ph, 1, k=3)
    assert abs(g[0, 1] - 0.5 * (math.cos(0.5) + math.cos(1.2))) < 1e-15
    assert abs(g[0, 0] - math.cos(0.5)) < 1e-15
    assert abs(g[0, 2] - math.cos(1.2)) < 1e-15


def test_phase_similarity_constant_field_and_invalid():
    rng = np.random.default_rng(4)
    N, oR, oC = 10, 9, 11
    ph = np.broadcast_to(rng.uniform(-3, 3, (N, 1, 1)), (N, oR, oC))
    flags = np.zeros((oR, oC), np.uint8)
    flags[4, 5] = O.FLAG_INVALID
    g = Q.phase_similarity(ph, 3, flags=flags)
    assert g[4, 5] == 0.0
    g[4, 5] = 1.0
    np.testing.assert_allclose(g, 1.0, atol=1e-14)
    # a per-image offset common to all pixels changes nothing
    g2 = Q.phase_similarity(ph + rng.uniform(-3, 3, (N, 1, 1)), 3, flags=flags)
    g2[4, 5] = 1.0
    np.testing.assert_allclose(g2, 1.0, atol=1e-14)


def test_phase_similarity_median_of_four_neighbours():
    """3 x 3 grid, radius 1 (the four edge neighbours), N = 2: similarities
    cos(d) for offsets d = 0.1, 0.4, 0.9, 2.0 at up, left, right, down."""
    ph = np.zeros((2, 3, 3))
    for (y, x), d in zip([(0, 1), (1, 0), (1, 2), (2, 1)], [0.1, 0.4, 0.9, 2.0]):
        ph[1, y, x] = d
    g = Q.phase_similarity(ph, 1)
    assert abs(g[1, 1] - 0.5 * (math.cos(0.4) + math.cos(0.9))) < 1e-15


# ---------------------------------------------------------------- PS selection and regridding
def test_amplitude_dispersion_closed_forms():
    rng = np.random.default_rng(5)
    ph = np.exp(1j * rng.uniform(-3, 3, (8, 2, 2)))
    amp = np.array([2.0, 4.0] * 4)[:, None, None] * np.ones((8, 2, 2))
    mean, var = O.amplitude_stats(amp * ph)
    ps, da = Q.ps_select(mean, var, 0.2)
    np.testing.assert_allclose(da, 1.0 / 3.0, rtol=1e-13)  # std 1, mean 3
    assert not ps.any()
    mean, var = O.amplitude_stats(np.full((5, 2, 2), 3 - 4j))
    ps, da = Q.ps_select(mean, var, 0.2)
    assert ps.all() and np.all(da < 1e-7)
    ps, da = Q.ps_select(np.zeros((1, 1)), np.zeros((1, 1)), 0.2)
    assert not ps.any() and np.isinf(da).all()


def test_regrid_cases_of_the_supplement():
    """Output blocks of 6 x 3 pixels: no PS -> the DS phasor; one PS -> its
    single-reference phase; two PS -> the lower D_A; a tie -> the first in
    row-major order; the ragged last column belongs to the last block."""
    rng = np.random.default_rng(6)
    N, R, C, w, ref = 4, 6, 13, (1, 1, 6, 3), 1
    z = rng.normal(size=(N, R, C)) + 1j * rng.normal(size=(N, R, C))
    oR, oC = R // 3, C // 6
    ds = np.exp(1j * rng.uniform(-3, 3, (N, oR, oC)))
    ps = np.zeros((R, C), bool)
    da = np.full((R, C), np.inf)
    ps[1, 8], da[1, 8] = True, 0.15            # block (0, 1): one PS
    ps[3, 2], da[3, 2] = True, 0.10            # block (1, 0): two PS
    ps[5, 4], da[5, 4] = True, 0.05
    ps[4, 7], da[4, 7] = True, 0.12            # block (1, 1): a tie, and the ragged column 12
    ps[3, 12], da[3, 12] = True, 0.12
    out, src = Q.regrid_ps_ds(z, ref, ds, ps, da, w)
    assert src[0, 0] == -1 and np.array_equal(out[:, 0, 0], ds[:, 0, 0])
    assert src[0, 1] == 1 * C + 8 and src[1, 0] == 5 * C + 4 and src[1, 1] == 3 * C + 12
    for (by, bx), (y, x) in [((0, 1), (1, 8)), ((1, 0), (5, 4)), ((1, 1), (3, 12))]:
        want = np.exp(1j * (np.angle(z[:, y, x]) - np.angle(z[ref, y, x])))
        np.testing.assert_allclose(out[:, by, bx], want, atol=1e-12)
        assert out[ref, by, bx] == 1.0


# ---------------------------------------------------------------- L1 network inversion
def test_incidence_matrix_reproduces_differences():
    N = 9
    A = Q.incidence_matrix(N, 3)
    x = np.arange(1.0, N) ** 1.5  # x_0 = 0 is the reference date
    full = np.concatenate([[0.0], x])
    for j, (a, b) in enumerate(Q.nearest_network(N, 3)):
        assert abs((A @ x)[j] - (full[b] - full[a])) < 1e-12
    assert np.linalg.matrix_rank(A) == N - 1


def test_soft_threshold_closed_form():
    np.testing.assert_array_equal(Q.soft_threshold([-3.0, -0.5, 0.0, 0.4, 2.5], 1.0), [-2.0, 0.0, 0.0, 0.0, 1.5])


def test_admm_recovers_consistent_series_and_sparse_unwrapping_errors():
    rng = np.random.default_rng(7)
    N = 15
    A = Q.incidence_matrix(N, 3)
    x = np.cumsum(rng.normal(0, 1.5, (N - 1, 6)), axis=0)
    b = A @ x
    np.testing.assert_allclose(Q.l1_invert_admm(A, b, rho=1.0, iters=300), x, atol=1e-6)
    # two interferograms off by whole cycles: the L1 solution ignores them
    e = np.zeros_like(b)
    e[5, :] = 2 * np.pi
    e[20, :] = -2 * np.pi
    np.testing.assert_allclose(Q.l1_invert_admm(A, b + e, rho=1.0, iters=3000), x, atol=1e-6)


def test_admm_reaches_the_linear_programme_optimum():
    """min ||A x - b||_1 as a linear programme (HiGHS) for noisy data: the
    ADMM objective matches the LP optimum."""
    rng = np.random.default_rng(8)
    N = 12
    A = Q.incidence_matrix(N, 3)
    M, n = A.shape
    for _ in range(3):
        b = A @ rng.normal(0, 2, n) + rng.normal(0, 0.3, M)
        b[rng.integers(M)] += 2 * np.pi
        c = np.concatenate([np.zeros(n), np.ones(M)])
        Aub = np.block([[A, -np.eye(M)], [-A, -np.eye(M)]])
        lp = linprog(c, A_ub=Aub, b_ub=np.concatenate([b, -b]), bounds=[(None, None)] * n + [(0, None)] * M,
                     method="highs")
        assert lp.status == 0
        x = Q.l1_invert_admm(A, b, rho=1.0, iters=20000)[:, 0]
        assert np.abs(A @ x - b).sum() <= lp.fun * (1 + 1e-6) + 1e-9


# ---------------------------------------------------------------- sequential scheme options
def _const_amp_batches(T, M, seed):
    rng = np.random.default_rng(seed)
    amp = np.ones((T, 3, 3))
    amp[:, 0, 0] = 1.6                 # q1, bit 0
    amp[0, 0, 2] = 3.0                 # q2, bit 2
    amp[1:3, 2, 0] = 2.0               # q3, bit 6
    amp[3, 2, 2] = 3.0                 # q4, bit 8
    return [amp[k][None] * np.exp(1j * rng.uniform(-np.pi, np.pi, (M, 3, 3))) for k in range(T)]


def test_sequential_exponential_weights_by_hand():
    """decay 0.5 at mini-stack 3 with K = 2: weights M (0.25, 0.5, 1) for
    mini-stacks 1, 2, 3, n_eff = 26.25, pooled scale ratios (constant
    amplitude within each mini-stack) q1 2.56 -> T = 11.19 (not an SHP),
    q2 1 -> SHP, q3 (0.25*4 + 0.5*4 + 1)/1.75 = 2.2857 -> T = 8.72 (SHP,
    unlike with even weights), q4 (0.25 + 0.5 + 9)/1.75 -> not."""
    M = 15
    out = O.sequential(_const_amp_batches(4, M, 16), 2, (1, 1, 3, 3), 1e-3, decay=0.5)
    assert abs(out[3]["n_eff"] - 26.25) < 1e-12
    bits = O.mask_bits(out[3]["mask"], (1, 1, 3, 3))[0, 0]
    assert (bits[0], bits[2], bits[6], bits[8]) == (False, True, True, False)
    thr = O.glrt_threshold(1e-3)
    t = lambda r, n: 2 * n * math.log((1 + r) ** 2 / (4 * r))
    assert t(2.56, 26.25) > thr and t(4 / 1.75, 26.25) < thr and t(9.75 / 1.75, 26.25) > thr
    even = O.sequential(_const_amp_batches(4, M, 16), 2, (1, 1, 3, 3), 1e-3)
    assert not O.mask_bits(even[3]["mask"], (1, 1, 3, 3))[0, 0][6]


def test_sequential_last_per_ministack_reference():
    """Supplement (compressed SLC strategy for separate batched processing):
    each compressed SLC carries the phase of the last real SLC of its
    mini-stack, so mini-stack k >= 1 is linked relative to the last date of
    mini-stack k - 1 (mini-stack 0 to its first date)."""
    M, K, R, C, w, T = 5, 2, 9, 9, (1, 1, 3, 3), 4
    rng = np.random.default_rng(17)
    phi = np.broadcast_to(np.cumsum(rng.uniform(-1, 1, (T * M, 1, 1)), axis=0), (T * M, R, C))
    s = rng.normal(size=(R, C)) + 1j * rng.normal(size=(R, C))
    z = np.exp(1j * phi) * s[None]
    out = O.sequential([z[i * M:(i + 1) * M] for i in range(T)], K, w, 1e-3, reference="last")
    cy, cx = O.output_centres(R, C, w)
    for k, o in enumerate(out):
        base = phi[0] if k == 0 else phi[k * M - 1]
        truth = phi[k * M:(k + 1) * M][:, cy][:, :, cx] - base[cy][:, cx][None]
        assert np.abs(O.wrap(np.angle(o["phasor"]) - truth)).max() < 1e-9, k
        # the compressed SLC has the phase of the mini-stack's last date
        last = z[(k + 1) * M - 1]
        assert np.abs(O.wrap(np.angle(o["kappa"] * np.conj(last)))).max() < 1e-9, k
