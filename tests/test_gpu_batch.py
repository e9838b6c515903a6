"""Batched, graph-replayed runs over mini-stacks with uneven N (the k-th
mini-stack of a burst carries k compressed SLCs, so N = 15 + k), as one
persistent launch (the default) and as one launch per stage, against the
single-call entry points (bit-identical: the same kernel bodies) and, item by
item, against the FP64 oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle import plink_oracle as O
from phase_parity import EPS, check_phases, coherence_error, phase_errors, sensitivity

pytestmark = pytest.mark.gpu

WINDOW = (11, 5, 6, 3)
SPECS = [  # (rows, cols, compressed SLCs): N = 15 + k, every grid ragged against the tiles
    (96, 390, 0),
    (150, 300, 2),
    (99, 384, 5),
    (120, 258, 7),
]


def _stacks(seed):
    out = []
    for i, (R, C, k) in enumerate(SPECS):
        wl = synth.Workload(f"batch{i}", R, C, 15, k, WINDOW, model="burst")
        out.append((wl, synth.make_stack(wl, seed=seed + i, device="cuda")))
    return out


def _single(plink, wl, z, prec, stats=None, n_eff=None):
    mean, var = stats if stats is not None else plink.amplitude_stats(z[wl.n_comp:].contiguous())
    mask, _ = plink.shp_select(mean, var, n_eff or wl.n_new, wl.window, wl.alpha)
    coh = plink.estimate_coherence(z, mask, wl.window, precision=prec)
    ph, _, fl = plink.phase_link(coh, ref=max(0, wl.n_comp - 1))
    oR, oC = wl.out_shape
    kap = plink.compress_ministack(z, wl.n_comp, wl.window, ph.view(wl.N, oR, oC))
    return ph.view(wl.N, oR, oC), fl, kap


def _items(stacks, stats1):
    items = []
    for i, (wl, z) in enumerate(stacks):
        it = dict(stack=z, first_real=wl.n_comp, ref=max(0, wl.n_comp - 1))
        if i == 1:  # supplied (e.g. merged) statistics with their own sample count
            it.update(mean=stats1[0], var=stats1[1], n_eff=45.0)
        items.append(it)
    return items


def _check_same(plink, b, stacks, prec, stats1):
    for i, (wl, z) in enumerate(stacks):
        ph, fl, kap = _single(plink, wl, z, prec, *( (stats1, 45.0) if i == 1 else (None, None) ))
        assert torch.equal(b.phasors[i], ph), f"item {i} phasors"
        assert torch.equal(b.flags[i], fl), f"item {i} flags"
        assert torch.equal(b.kappa[i], kap), f"item {i} kappa"


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("tune", [False, True])
def test_batch_matches_single_calls_and_replays(gpu_lib, prec, tune):
    plink = gpu_lib
    stacks = _stacks(seed=40)
    wl1, z1 = stacks[1]
    stats1 = plink.amplitude_stats(z1[wl1.n_comp:].contiguous())
    b = plink.Batch(_items(stacks, stats1), WINDOW, precision=prec, autotune=tune)
    print(b.describe(), flush=True)
    for rep in range(3):
        b.run()
        torch.cuda.synchronize()
        _check_same(plink, b, stacks, prec, stats1)
        # refill every input in place with new data; eager work between replays
        fresh = _stacks(seed=100 + 10 * rep)
        for (wl, z), (_, znew) in zip(stacks, fresh):
            z.copy_(znew)
        s1 = plink.amplitude_stats(z1[wl1.n_comp:].contiguous())
        stats1[0].copy_(s1[0])
        stats1[1].copy_(s1[1])
        torch.cuda.synchronize()
    assert "graph captured" in b.describe()
    b.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_items_against_oracle(gpu_lib, prec):
    """Every item of a batch (N = 15, 17, 20, 22: one per linking-kernel
    class of the sequential batched workload) against the FP64 oracle; the
    coherence the criterion needs comes from the single-call path, which the
    batch reproduces bit for bit (test above)."""
    plink = gpu_lib
    stacks = _stacks(seed=60)
    b = plink.Batch([dict(stack=z, first_real=wl.n_comp, ref=max(0, wl.n_comp - 1)) for wl, z in stacks],
                    WINDOW, precision=prec)
    b.run()
    torch.cuda.synchronize()
    for i, (wl, z) in enumerate(stacks):
        ref = max(0, wl.n_comp - 1)
        r = O.link_ministack(z.cpu().numpy(), wl.n_comp, wl.window, wl.alpha, ref)
        mean, var = plink.amplitude_stats(z[wl.n_comp:].contiguous())
        mask, _ = plink.shp_select(mean, var, wl.n_new, wl.window, wl.alpha)
        np.testing.assert_array_equal(mask.cpu().numpy().view(np.uint32), r["mask"])
        coh = plink.estimate_coherence(z, mask, wl.window, precision=prec).cpu().numpy()
        dC, dmax = coherence_error(coh, r["coh"])
        assert dmax <= EPS[prec]
        ph = b.phasors[i].cpu().numpy().reshape(wl.N, -1)
        err = phase_errors(ph, r["link"]["phasor"])
        check_phases(f"batch item {i} (N={wl.N}, {wl.R}x{wl.C})", err, sensitivity(r["coh"], ref),
                     b.flags[i].cpu().numpy(), r["link"], prec, r["coh"], dC_pix=dC, min_well_posed=len(dC) // 10)
        kap = O.compress(z.cpu().numpy(), wl.n_comp, b.phasors[i].cpu().numpy(), wl.window)
        scale = np.abs(z[wl.n_comp:].cpu().numpy()).astype(np.float64).sum(0)
        assert np.max(np.abs(b.kappa[i].cpu().numpy() - kap) / scale) <= 1e-6
    b.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_chained_sequence_matches_sequential_driver(gpu_lib, prec):
    """The sequential scheme of two bursts as one plan: level k holds
    mini-stack k of both bursts, whose compressed planes are the kappa
    buffers written by levels < k.  One graph run equals pushing the
    mini-stacks through the sequential driver, bit for bit."""
    plink = gpu_lib
    Kmax, n = 2, 4  # the window of compressed SLCs slides
    bursts = []
    for bi in range(2):
        wl = synth.crop("sequential", 96, 198 if bi == 0 else 252)
        bursts.append((wl, synth.make_sequence(wl, seed=70 + bi, ministacks=n).cuda()))
    items, kappas, stats = [], {}, {}
    for bi, (wl, z) in enumerate(bursts):
        M = wl.n_new
        for k in range(n):
            stats[bi, k] = plink.amplitude_stats(z[k * M:(k + 1) * M].contiguous())
            kappas[bi, k] = torch.empty((wl.R, wl.C), dtype=torch.complex64, device="cuda")
    for bi, (wl, z) in enumerate(bursts):
        M = wl.n_new
        for k in range(n):
            K = min(k, Kmax)
            groups = [stats[bi, j] for j in range(k - K, k + 1)]
            mean, var = plink.merge_amplitude_stats(torch.stack([g[0] for g in groups]),
                                                    torch.stack([g[1] for g in groups]), [M] * len(groups))
            planes = [kappas[bi, j] for j in range(k - K, k)] + [z[k * M + m] for m in range(M)]
            items.append(dict(planes=planes, first_real=K, ref=max(0, K - 1), mean=mean, var=var,
                              n_eff=float((K + 1) * M), kappa=kappas[bi, k], level=k))
    b = plink.Batch(items, bursts[0][0].window, precision=prec, autotune=True)
    print(b.describe(), flush=True)
    assert "mode single launch" in b.describe() and "launches per run 1" in b.describe()
    b.run()
    b.check()  # no wait of the single launch ran past its bound
    torch.cuda.synchronize()
    single = [(p.clone(), f.clone()) for p, f in zip(b.phasors, b.flags)]
    single_kappa = {key: v.clone() for key, v in kappas.items()}
    # the same plan as one launch per stage and kernel variant: the same bits
    b.set_single_launch(False)
    b.run()
    torch.cuda.synchronize()
    assert "mode stage launches" in b.describe()
    for i, (p, f) in enumerate(single):
        assert torch.equal(b.phasors[i], p) and torch.equal(b.flags[i], f), f"item {i}: single launch differs"
    for key, v in single_kappa.items():
        assert torch.equal(kappas[key], v), f"kappa {key}: single launch differs"
    b.set_single_launch(True)
    for _ in range(2):  # replays of the single-launch graph keep the counters consistent
        b.run()
    b.check()
    torch.cuda.synchronize()
    for i, (p, f) in enumerate(single):
        assert torch.equal(b.phasors[i], p) and torch.equal(b.flags[i], f), f"item {i}: replay differs"
    it = iter(range(len(items)))
    for bi, (wl, z) in enumerate(bursts):
        M = wl.n_new
        seq = plink.Sequential(wl.R, wl.C, M, Kmax, wl.window, wl.alpha, precision=prec)
        for k in range(n):
            i = next(it)
            ph, kap, fl = seq.push(z[k * M:(k + 1) * M].contiguous(), want_flags=True)
            K = min(k, Kmax)
            assert torch.equal(b.phasors[i][K:], ph), f"burst {bi} mini-stack {k} phasors"
            assert torch.equal(b.flags[i], fl.reshape(-1)), f"burst {bi} mini-stack {k} flags"
            assert torch.equal(kappas[bi, k], kap), f"burst {bi} mini-stack {k} kappa"
        seq.close()
    b.close()


def test_single_launch_wait_bound_reports_and_recovers(gpu_lib):
    """The failure path of the single launch, forced from the host: with a
    wait bound of 0 every dependency wait gives up at once, the launch still
    ends and check() reports it (the outputs of that run are not used); with
    the bound restored the run matches the stage launches bit for bit."""
    plink = gpu_lib
    wl = synth.crop("sequential", 96, 198)
    z = synth.make_sequence(wl, seed=90, ministacks=3).cuda()
    M = wl.n_new
    kap = [torch.empty((wl.R, wl.C), dtype=torch.complex64, device="cuda") for _ in range(3)]
    items = []
    for k in range(3):
        K = min(k, 2)
        items.append(dict(planes=kap[k - K:k] + [z[k * M + m] for m in range(M)], first_real=K, ref=max(0, K - 1),
                          kappa=kap[k], level=k))
    b = plink.Batch(items, wl.window, precision="bf16")
    b.set_single_launch(False)
    b.run()
    torch.cuda.synchronize()
    ref = [p.clone() for p in b.phasors]
    b.set_single_launch(True)
    b.set_wait_limit(0)
    b.run()
    with pytest.raises(plink.PlinkError):
        b.check()
    b.set_wait_limit(1 << 20)
    b.run()
    b.check()
    torch.cuda.synchronize()
    for i, p in enumerate(ref):
        assert torch.equal(b.phasors[i], p), f"item {i}"
    b.close()
