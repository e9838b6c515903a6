"""The allocation-free fused entry point (pl_phase_link_fused_noalloc), called
through the C ABI, against pl_phase_link_fused with a caller workspace: two
calls in a row, the second on a smaller input, outputs bit-identical (both
run the same kernels on the same pixels; the band height does not change a
pixel's result).  The first input is as wide as the 4096 x 16384 workload,
so that its packed coherence (426 MB) passes through the 128 MiB buffer in
four bands while the workspace call takes one."""
import ctypes

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _inputs(plink, name, R, C, seed):
    wl = synth.crop(name, R, C)
    z = synth.make_stack(wl, seed=seed, device="cuda")
    mean, var = plink.amplitude_stats(z[wl.n_comp:].contiguous())
    mask, _ = plink.shp_select(mean, var, wl.n_new, wl.window, wl.alpha)
    return wl, z, mask


def _outputs(N, P, dev):
    return (torch.empty((N, P), dtype=torch.complex64, device=dev), torch.empty((N, P), dtype=torch.float32, device=dev),
            torch.empty((P,), dtype=torch.float32, device=dev), torch.empty((P,), dtype=torch.float32, device=dev),
            torch.empty((P,), dtype=torch.uint8, device=dev), torch.zeros((24,), dtype=torch.int64, device=dev))


def test_noalloc_matches_workspace_entry_point(gpu_lib):
    plink = gpu_lib
    lib = plink.load()
    P_ = ctypes.c_void_p
    for name, R, C, seed, prec in (("scale", 180, 16384, 91, 1), ("burst", 96, 390, 92, 0)):
        wl, z, mask = _inputs(plink, name, R, C, seed)
        oR, oC = wl.out_shape
        P = oR * oC
        ref = max(0, wl.n_comp - 1)
        stream = P_(torch.cuda.current_stream().cuda_stream)
        a = _outputs(wl.N, P, z.device)
        b = _outputs(wl.N, P, z.device)
        row, full = plink.phase_link_fused_workspace(wl.N, wl.R, wl.C, wl.window)
        ws = torch.empty((full,), dtype=torch.uint8, device="cuda")
        common = [P_(z.data_ptr()), wl.N, wl.R, wl.C, plink._win(wl.window), P_(mask.data_ptr()), prec, ref, 0]
        st = lib.pl_phase_link_fused(*common, *[P_(t.data_ptr()) for t in a], P_(ws.data_ptr()), full, stream)
        assert st == 0, lib.pl_last_error()
        st = lib.pl_phase_link_fused_noalloc(*common, *[P_(t.data_ptr()) for t in b], stream)
        assert st == 0, lib.pl_last_error()
        torch.cuda.synchronize()
        for x, y in zip(a, b):
            assert torch.equal(x, y), name
        assert np.all(np.abs(np.abs(a[0].cpu().numpy()) - 1) < 1e-5)
        print(f"[noalloc] {name} {wl.R}x{wl.C} N={wl.N}: identical to the workspace entry point", flush=True)
