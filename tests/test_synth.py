"""The seeded input generator: determinism and the workload's structure."""
import numpy as np
import torch

import synth
from oracle import plink_oracle as O


def test_same_seed_same_stack_different_seed_differs():
    a = synth.make_stack("tiny", seed=3)
    b = synth.make_stack("tiny", seed=3)
    c = synth.make_stack("tiny", seed=4)
    assert a.dtype == torch.complex64 and a.shape == (10, 64, 64)
    assert torch.equal(a, b)
    assert not torch.equal(a, c)


def test_land_cover_fractions_burst_model():
    wl = synth.crop("burst", 256, 512)
    amp, g0, ginf, cls = synth.land_cover(wl, 0, 0, torch.device("cpu"))
    frac = [(cls == k).float().mean().item() for k in range(3)]
    assert abs(frac[2] - 0.30) < 0.03   # water
    assert abs(frac[1] - 0.20) < 0.03   # persistent scatterers
    ds = cls == 0
    assert g0[ds].min() >= 0.3 and g0[ds].max() <= 0.9


def test_compressed_planes_carry_first_new_epoch_phase():
    """The analytic compressed planes share the reference phase of the first
    new epoch, so at PS pixels (coherence 0.98) their interferogram with it is
    near zero phase."""
    wl = synth.crop("scale", 64, 128)
    z, truth = synth.make_stack(wl, seed=1, with_truth=True)
    assert z.shape[0] == 25
    ps = truth["cls"] == 1
    ifg = (z[:10] * z[10].conj())[:, ps]
    assert torch.angle(ifg).abs().median() < 0.4


def test_sample_coherence_follows_model_at_full_window():
    """DS sample coherence decays with temporal baseline as the model says."""
    z, truth = synth.make_stack("tiny", seed=2, with_truth=True)
    zs = z.numpy()
    w = (5, 5, 8, 8)
    oR, oC = O.output_grid(64, 64, w)
    full = np.zeros((oR, oC, 4), np.uint32)
    for b in range(121):
        full[..., b // 32] |= np.uint32(1 << (b % 32))
    Cm, _ = O.coherence(zs, full, w)
    g1 = np.abs(Cm[:, 0, 1]).mean()
    g9 = np.abs(Cm[:, 0, 9]).mean()
    assert g1 > g9 + 0.1
