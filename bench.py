#!/usr/bin/env python3
"""Throughput of the phase-linking hot path on one MI355X.

One step = amplitude statistics -> GLRT SHP masks -> sample coherence ->
EMI/EVD phase linking -> compressed SLC over one synthetic mini-stack that is
already resident in HBM.  Prints one JSON line.

The headline is the mixed-precision workload at scale (4096 x 16384, N = 25:
10 compressed + 15 new SLCs, split-BF16 coherence); the plain FP32 path on
the 2048 x 8192, N = 15 burst is reported beside it, with the other
precision of each for the mixed/plain speed-up.  Each step is bracketed by
HIP events on the stream the kernels run on; ms_per_step is the median of
the fused step (coherence straight into linking through bands of packed
triangles), split_ms_per_step that of the step with one call per stage,
whose per-stage times give the roofline figures.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload scale|burst|tiny]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {  # MI355X published peaks
    "hbm_GBps": 8000.0,
    "bf16_mfma_TFLOPs": 2500.0,
    "fp32_mfma_TFLOPs": 157.3,
    "fp32_valu_TFLOPs": 78.6,  # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz, no packed FP32
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="scale")
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp32"])
    ap.add_argument("--no-compare", action="store_true", help="skip the other precision")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--only-main", action="store_true",
                    help="skip the other-workload, batched-sequence and adjoint legs")
    ap.add_argument("--only-sequence", action="store_true",
                    help="only the batched-sequence leg (4 bursts x 8 mini-stacks)")
    ap.add_argument("--skip-fused", action="store_true", help="do not time the fused coherence + linking step")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="oracle worker processes (default: the usable host cores, at most 16)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    return ap.parse_args()


class Path:
    """The hot path on one resident stack with pre-built geometry."""

    def __init__(self, plink, wl, stack, precision):
        self.plink, self.wl, self.z, self.prec = plink, wl, stack, precision
        self.ref = max(0, wl.n_comp - 1)
        self.first_real = wl.n_comp
        self.real = stack[wl.n_comp:] if wl.n_comp else stack

    def stats(self):
        return self.plink.amplitude_stats(self.real)

    def glrt(self, st):
        return self.plink.shp_select(st[0], st[1], self.wl.n_new, self.wl.window, self.wl.alpha)

    def coherence(self, m):
        return self.plink.estimate_coherence(self.z, m[0], self.wl.window, precision=self.prec)

    def link(self, coh):
        return self.plink.phase_link(coh, ref=self.ref)

    def compress(self, ln):
        oR, oC = self.wl.out_shape
        return self.plink.compress_ministack(self.z, self.first_real, self.wl.window,
                                             ln[0].view(self.wl.N, oR, oC))

    def step(self):
        st = self.stats()
        m = self.glrt(st)
        coh = self.coherence(m)
        ln = self.link(coh)
        k = self.compress(ln)
        return m, coh, ln, k

    def fused(self, m, ws):
        return self.plink.phase_link_fused(self.z, m[0], self.wl.window, self.ref, self.prec, workspace=ws)

    def step_fused(self, ws):
        st = self.stats()
        m = self.glrt(st)
        ln = self.fused(m, ws)
        k = self.compress(ln)
        return m, ln, k


def time_steps(torch, fn, steps, warmup):
    """Median and mean device time of one step (ms): W untimed steps, then
    exactly K steps, each between two HIP events on the current stream,
    with the device synchronised before and after."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for i in range(steps):
        fn()
        ev[i + 1].record()
    torch.cuda.synchronize()
    per = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
    mid = steps // 2
    median = per[mid] if steps % 2 else 0.5 * (per[mid - 1] + per[mid])
    return {"median": median, "mean": ev[0].elapsed_time(ev[steps]) / steps, "min": per[0], "max": per[-1]}


def stage_times(torch, path, steps):
    """Median device time of each stage, HIP events on the stream the kernels use."""
    names = ["stats", "glrt", "coherence", "link", "compress"]
    acc = {n: [] for n in names}
    for _ in range(steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
        ev[0].record()
        st = path.stats(); ev[1].record()
        m = path.glrt(st); ev[2].record()
        coh = path.coherence(m); ev[3].record()
        ln = path.link(coh); ev[4].record()
        path.compress(ln); ev[5].record()
        torch.cuda.synchronize()
        for i, n in enumerate(names):
            acc[n].append(ev[i].elapsed_time(ev[i + 1]))
    return {n: sorted(v)[len(v) // 2] for n, v in acc.items()}


def algorithmic(wl, shp_sum, P, prec):
    """Algorithmic bytes and flops of each stage (one launch each) and the
    peak each is measured against.  Coherence bytes count the output as the
    packed Hermitian triangle (its N(N+1)/2 unique entries); linking counts
    2 N^3 FP64 flops (the |C| inverse) and (8/3) N^3 + 80 N^2 FP32 flops (a
    complex factorisation and ten mat-vec-sized solves) per pixel against the
    vector ALU peak of 78.6 TFLOP/s, which FP32 and FP64 share when packed
    FP32 instructions are not used."""
    R, C, N, M = wl.R, wl.C, wl.N, wl.n_new
    nw = ((2 * wl.window[0] + 1) * (2 * wl.window[1] + 1) + 31) // 32
    px = R * C
    tri = N * (N + 1) // 2
    mfma_peak = PEAK["bf16_mfma_TFLOPs"] if prec == "bf16" else PEAK["fp32_mfma_TFLOPs"]
    link64 = 2 * N ** 3
    link32 = (8 * N ** 3) / 3 + 80 * N ** 2
    return {
        "stats": {"bytes": px * M * 8 + px * 16},
        "glrt": {"bytes": px * 16 + P * nw * 4 + P * 2},
        # complex MACs over the N(N+1)/2 unique entries of each Hermitian A,
        # 8 flops each, over the pixel's SHPs
        "coherence": {"bytes": px * N * 8 + P * nw * 4 + P * tri * 8,
                      "flops": shp_sum * tri * 8, "flop_peak": mfma_peak, "flop_bound": "mfma"},
        "link": {"bytes": P * tri * 8 + P * N * 8,
                 "flops": P * (link64 + link32), "flop_peak": PEAK["fp32_valu_TFLOPs"], "flop_bound": "alu",
                 "flops_fp64": P * link64, "flops_fp32": P * link32},
        "compress": {"bytes": px * M * 8 + P * N * 8 + px * 8},
    }


def roofline(alg, t_ms):
    """The binding resource of a stage: the larger of its ideal HBM time and
    its ideal compute time at the published peaks."""
    t = t_ms * 1e-3
    t_hbm = alg["bytes"] / (PEAK["hbm_GBps"] * 1e9)
    t_flop = alg["flops"] / (alg["flop_peak"] * 1e12) if "flops" in alg else 0.0
    if t_flop > t_hbm:
        r = {"bound": alg["flop_bound"], "achieved": alg["flops"] / t / 1e12,
             "peak": alg["flop_peak"], "unit": "TFLOP/s"}
    else:
        r = {"bound": "hbm", "achieved": alg["bytes"] / t / 1e9, "peak": PEAK["hbm_GBps"],
             "unit": "GB/s"}
    r["frac"] = r["achieved"] / r["peak"]
    return r


def kernel_name(stage, wl, prec):
    """Device kernel that runs a stage (as rocprofv3 names it, without spaces)."""
    tile = 16 if wl.N <= 16 else 32
    rows = 1 if wl.N <= 16 else 2          # rows per lane of the linking kernel's 16-lane groups
    cols = max(12, 4 * ((wl.N + 3) // 4))  # columns per row of the linking kernel
    return {"stats": "amp_stats_vec", "glrt": "glrt_kernel",
            "coherence": f"coherence_kernel<{tile},{'true' if prec == 'bf16' else 'false'}>",
            "link": f"phase_link_kernel<{rows},{cols}>", "compress": "compress_kernel"}[stage]


def _code_text(path):
    """A C++ source with its comments and blank lines removed, so that a
    comment edit does not count as a kernel change.  (The kernel sources
    hold no comment markers inside string literals.)"""
    import re
    text = open(path, encoding="utf-8").read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip()).encode()


def source_hash(name):
    """sha256 prefix of a kernel source file's code together with the
    package's device headers (the kernels include them), or None if it is
    missing."""
    import glob
    import hashlib
    csrc = os.path.join(ROOT, "paper_2511_12051_amd", "csrc")
    path = os.path.join(csrc, name)
    if not os.path.exists(path):
        return None
    h = hashlib.sha256(_code_text(path))
    for hdr in sorted(glob.glob(os.path.join(csrc, "*.hpp"))):
        h.update(_code_text(hdr))
    return h.hexdigest()[:16]


def measured_traffic(kernel, wl, prec):
    """HBM bytes per launch of a kernel from the FETCH_SIZE / WRITE_SIZE
    summary under profiles/ (already scaled by the copy calibration), or None
    when there is none for this workload or the kernel source has changed
    since the counters were taken."""
    import glob
    import hashlib
    for f in glob.glob(os.path.join(ROOT, "profiles", f"hbm_traffic_{wl.name}_*.txt")):
        for line in open(f):
            if not line.startswith("traffic "):
                continue
            kv = dict(t.split("=", 1) for t in line.split()[1:])
            if kv.get("kernel") != kernel or kv.get("precision") != prec:
                continue
            if source_hash(kv["source"]) != kv["sha256"]:
                return None
            return float(kv["fetch_bytes"]) + float(kv["write_bytes"])
    return None


def _oracle_band(args):
    """One worker of the CPU baseline: the oracle on a band of output rows,
    on its own crop that holds every window of the band; with `sens`, also
    the phase sensitivity of the band's pixels (test infrastructure, outside
    the timed run)."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    from oracle import plink_oracle as O
    z, first_real, window, alpha, ref, skip, rows, sens = args
    r = O.link_ministack(z, first_real, window, alpha, ref)
    oR, oC = O.output_grid(z.shape[1], z.shape[2], window)
    sl = slice(skip * oC, (skip + rows) * oC)
    out = (r["link"]["phasor"][:, sl], r["link"]["flag"][sl], r["link"]["min_pivot"][sl],
           r["coh"][sl].astype("complex64"))
    if sens:
        out += (O.phase_sensitivity(r["coh"][sl], ref=ref, n_probe=8),)
    return out


def cpu_baseline(wl_name, seed, workers=0):
    """The FP64 oracle on a bounded crop of the same workload, split into
    bands of output rows over a pool of worker processes (one per usable host
    core, at most 16).  Returns the baseline record and the oracle's results
    on the crop (for the per-result error of the GPU path)."""
    import multiprocessing as mp

    import numpy as np

    import synth
    R, C = (64, 64) if wl_name == "tiny" else (576, 1536)
    wl = synth.crop(wl_name, R, C)
    z = synth.make_stack(wl, seed=seed).numpy()
    hx, hy, sx, sy = wl.window
    oR, oC = wl.out_shape
    ncore = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    workers = workers or min(16, ncore)
    nb = min(oR, workers)
    bounds = [(oR * i) // nb for i in range(nb + 1)]
    jobs = []
    for a, b in zip(bounds[:-1], bounds[1:]):
        # the band's crop starts at a whole stride (so that its output grid
        # lines up with the full one) at or above the first window row of
        # output row a, and ends past the last window row of output row b - 1
        y0 = max(0, ((a * sy + sy // 2 - hy) // sy) * sy)
        y1 = min(R, max(b * sy, (b - 1) * sy + sy // 2 + hy + 1))
        jobs.append((np.ascontiguousarray(z[:, y0:y1]), wl.n_comp, wl.window, wl.alpha, max(0, wl.n_comp - 1),
                     a - y0 // sy, b - a, False))
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        # start-up and imports, untimed; a bounded wait, so that workers that
        # fail to start end the run instead of hanging it
        pool.map_async(_oracle_band, jobs[:workers]).get(timeout=900)
        t0 = time.perf_counter()
        pool.map_async(_oracle_band, jobs).get(timeout=900)
        wall = time.perf_counter() - t0
        # again with the sensitivities the accuracy report needs (untimed)
        parts = pool.map_async(_oracle_band, [j[:-1] + (True,) for j in jobs]).get(timeout=900)
    res = {"phasor": np.concatenate([p[0] for p in parts], axis=1), "flag": np.concatenate([p[1] for p in parts]),
           "min_pivot": np.concatenate([p[2] for p in parts]), "coh": np.concatenate([p[3] for p in parts]),
           "sens": np.concatenate([p[4] for p in parts])}
    P = oR * oC
    rec = {"value": P / wall, "unit": "pixels/s", "cores": workers, "kind": "oracle",
           "sample": f"{wl.R}x{wl.C} crop of the {wl_name} workload (N={wl.N}, window {wl.window}), "
                     f"{P} output pixels in {nb} bands of output rows over {workers} processes, "
                     f"{wall:.1f} s wall; host reports {ncore} usable cores"}
    return rec, wl, z, res


def accuracy_vs_oracle(torch, plink, wl, z, orc):
    """Per-result error of the GPU path against the oracle on the baseline
    crop: coherence (max |dC|) and linked phases (wrapped error percentiles
    over valid pixels, and the maximum over the pixels the oracle marks well
    posed: 3 x phase sensitivity x the path's coherence error bound
    <= 1e-3 rad, the criterion of the parity tests)."""
    import numpy as np
    from oracle import plink_oracle as O
    out = {"crop": f"{wl.R}x{wl.C}", "pixels": int(len(orc["flag"]))}
    zc = torch.from_numpy(z).cuda()
    ref = max(0, wl.n_comp - 1)
    mean, var = plink.amplitude_stats(zc[wl.n_comp:].contiguous())
    mask, _ = plink.shp_select(mean, var, wl.n_new, wl.window, wl.alpha)
    for prec in ("bf16", "fp32"):
        coh = plink.estimate_coherence(zc, mask, wl.window, precision=prec)
        ph, lam, flags = plink.phase_link(coh, ref=ref)
        torch.cuda.synchronize()
        C = coh.cpu().numpy()
        okc = np.all(np.isfinite(orc["coh"].reshape(len(C), -1)), axis=1)
        dC = float(np.abs(C[okc].astype(np.complex128) - orc["coh"][okc].astype(np.complex128)).max())
        err = np.abs(np.angle(ph.cpu().numpy().astype(np.complex128) * np.conj(orc["phasor"]))).max(axis=0)
        fl = flags.cpu().numpy()
        valid = (fl == orc["flag"]) & (orc["flag"] != O.FLAG_INVALID)
        eps = 3e-5 if prec == "bf16" else 2.5e-6
        wp = valid & (3.0 * orc["sens"] * eps <= 1e-3)
        out[prec] = {"max_abs_dC": dC, "phase_err_p50": float(np.percentile(err[valid], 50)),
                     "phase_err_p99": float(np.percentile(err[valid], 99)),
                     "phase_err_max_well_posed": float(err[wp].max()) if wp.any() else None,
                     "well_posed_frac": float(wp.mean()), "flag_mismatch": int((fl != orc["flag"]).sum())}
    return out


def measure(torch, plink, wl, stack, prec, steps, warmup, skip_fused=False):
    """ms/step (median), per-stage ms, solver counters and SHP total of the
    single-call path at one precision."""
    import numpy as np
    oR, oC = wl.out_shape
    P = oR * oC
    path = Path(plink, wl, stack, prec)
    print(f"[bench] {wl.name} {prec}: warmup {warmup}, steps {steps}", file=sys.stderr, flush=True)
    t = time_steps(torch, path.step, steps, warmup)
    stages = stage_times(torch, path, max(3, steps // 2))
    m, coh, ln, k = path.step()
    cnt = plink.new_counters()
    plink.phase_link(coh, ref=path.ref, counters=cnt)
    torch.cuda.synchronize()
    cnt = dict(zip(plink.COUNTERS, cnt.cpu().tolist()))
    shp_sum = int(m[1].to(torch.int32).sum().item())
    flags = ln[2].cpu().numpy()
    del m, coh, ln, k
    print(f"[bench] {wl.name} {prec}: {t['median']:.3f} ms/step (median), stages "
          f"{json.dumps({k: round(v, 4) for k, v in stages.items()})}", file=sys.stderr, flush=True)
    if skip_fused:
        return {"ms": t["median"], "ms_mean": t["mean"], "ms_min": t["min"], "ms_max": t["max"], "stages": stages,
                "fused": None, "shp_sum": shp_sum, "value": P / (t["median"] * 1e-3),
                "evd_frac": float(np.mean(flags == 1)), "invalid_frac": float(np.mean(flags == 2)),
                "link_counters": {"iters_per_pixel": cnt["iters"] / P,
                                  "shift_retries_per_pixel": cnt["shift_retry"] / P,
                                  "not_converged": cnt["not_converged"], "glrt_band_pairs": cnt["glrt_band"]}}
    # the same step with coherence and linking fused through a bounded buffer
    # of packed coherence bands (whole rows)
    row, full = plink.phase_link_fused_workspace(wl.N, wl.R, wl.C, wl.window)
    # at most 16 GiB of band buffer: every output row of the 4096x16384 N=25
    # workload (9.7 GB of packed coherence) fits in one band
    cap = int(os.environ.get("PLINK_FUSED_BUFFER_GIB", "16")) << 30
    ws = torch.empty((min(full, max(row, cap // row * row)),), dtype=torch.uint8, device=stack.device)
    tf = time_steps(torch, lambda: path.step_fused(ws), steps, warmup)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    m = path.glrt(path.stats())
    fused_ms = []
    for _ in range(max(3, steps // 2)):
        ev[0].record()
        path.fused(m, ws)
        ev[1].record()
        torch.cuda.synchronize()
        fused_ms.append(ev[0].elapsed_time(ev[1]))
    fused = {"ms_per_step": tf["median"], "value": P / (tf["median"] * 1e-3),
             "fused_stage_ms": sorted(fused_ms)[len(fused_ms) // 2], "workspace_bytes": ws.numel(),
             "rows_per_band": ws.numel() // row}
    del ws, m
    print(f"[bench] {wl.name} {prec} fused: {tf['median']:.3f} ms/step, fused stage {fused['fused_stage_ms']:.3f} ms",
          file=sys.stderr, flush=True)
    return {"ms": t["median"], "ms_mean": t["mean"], "ms_min": t["min"], "ms_max": t["max"], "stages": stages,
            "fused": fused,
            "shp_sum": shp_sum, "value": P / (t["median"] * 1e-3),
            "evd_frac": float(np.mean(flags == 1)), "invalid_frac": float(np.mean(flags == 2)),
            "link_counters": {"iters_per_pixel": cnt["iters"] / P, "shift_retries_per_pixel": cnt["shift_retry"] / P,
                              "not_converged": cnt["not_converged"], "glrt_band_pairs": cnt["glrt_band"]}}


def describe(wl):
    oR, oC = wl.out_shape
    return (f"{wl.name}: {wl.R}x{wl.C} grid, N={wl.N} ({wl.n_comp} compressed + {wl.n_new} new), "
            f"half-window {wl.window[0]}x{wl.window[1]}, stride {wl.window[2]}x{wl.window[3]}, "
            f"{oR * oC} output pixels")


def stage_rooflines(wl, r, prec):
    oR, oC = wl.out_shape
    alg = algorithmic(wl, r["shp_sum"], oR * oC, prec)
    return alg, {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in roofline(alg[k], v).items()}
                 for k, v in r["stages"].items()}


def leg_other(torch, plink, synth, args, name, steps, warmup):
    """Another workload at both precisions (plain FP32 first when it is the
    burst, whose configuration is the plain path)."""
    wl = synth.WORKLOADS[name]
    print(f"[bench] generating {wl.name} {wl.N}x{wl.R}x{wl.C}", file=sys.stderr, flush=True)
    stack = synth.make_stack(wl, seed=args.seed, device="cuda")
    out = {"workload": describe(wl)}
    for prec in ("fp32", "bf16"):
        r = measure(torch, plink, wl, stack, prec, steps, warmup, args.skip_fused)
        _, sr = stage_rooflines(wl, r, prec)
        out[prec] = {"value": r["value"], "unit": "pixels/s", "ms_per_step": r["ms"], "ms_per_step_mean": r["ms_mean"],
                     "stage_ms": {k: round(v, 4) for k, v in r["stages"].items()}, "stage_roofline": sr,
                     "link_counters": r["link_counters"], "fused_path": r["fused"]}
    out["mixed_speedup_vs_fp32"] = out["fp32"]["ms_per_step"] / out["bf16"]["ms_per_step"]
    del stack
    torch.cuda.empty_cache()
    return out


def leg_sequence(torch, plink, synth, args, prec):
    """Sequential batched: 4 bursts of 1024x4096, 8 mini-stacks of 15 SLCs each
    (N = 15..22), every burst and mini-stack in one graph-replayed plan; the
    same work pushed through the sequential driver for comparison."""
    wl = synth.WORKLOADS["sequential"]
    M, n, Kmax = wl.n_new, wl.ministacks, wl.ministacks - 1
    oR, oC = wl.out_shape
    print(f"[bench] generating {wl.bursts} bursts x {n * M} epochs of {wl.R}x{wl.C}", file=sys.stderr, flush=True)
    seqs = [synth.make_sequence(wl, seed=args.seed, device="cuda", burst=b) for b in range(wl.bursts)]
    items = []
    for b, z in enumerate(seqs):
        st = [plink.amplitude_stats(z[k * M:(k + 1) * M].contiguous()) for k in range(n)]
        kap = [torch.empty((wl.R, wl.C), dtype=torch.complex64, device="cuda") for _ in range(n)]
        for k in range(n):
            K = min(k, Kmax)
            g = st[k - K:k + 1]
            mean, var = plink.merge_amplitude_stats(torch.stack([x[0] for x in g]), torch.stack([x[1] for x in g]),
                                                    [M] * len(g))
            items.append(dict(planes=kap[k - K:k] + [z[k * M + m] for m in range(M)], first_real=K,
                              ref=max(0, K - 1), mean=mean, var=var, n_eff=float((K + 1) * M), kappa=kap[k],
                              level=k))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch = plink.Batch(items, wl.window, wl.alpha, precision=prec, autotune=True)
    plan_s = time.perf_counter() - t0
    batch.run()  # captures the graph (one persistent launch per run)
    ms = time_steps(torch, batch.run, 10, 3)["median"]
    batch.check()
    desc = batch.describe()
    # the same plan as one launch per stage and kernel variant
    batch.set_single_launch(False)
    batch.run()
    ms_stages = time_steps(torch, batch.run, 10, 3)["median"]
    launches_stages = int(batch.describe().strip().splitlines()[-1].split()[-1])
    batch.set_single_launch(True)

    def driver():
        for z in seqs:
            s = plink.Sequential(wl.R, wl.C, M, Kmax, wl.window, wl.alpha, precision=prec)
            for k in range(n):
                s.push(z[k * M:(k + 1) * M])
            s.close()

    ms_driver = time_steps(torch, driver, 3, 1)["median"]
    batch.close()
    px = wl.bursts * n * oR * oC
    return {"workload": f"{wl.bursts} bursts x {n} mini-stacks of {M} SLCs, {wl.R}x{wl.C}, N=15..22, "
                        f"half-window {wl.window[0]}x{wl.window[1]}, stride {wl.window[2]}x{wl.window[3]}",
            "precision": prec, "value": px / (ms * 1e-3), "unit": "pixels/s", "ms_per_run": ms,
            "output_pixels": px, "driver_ms": ms_driver, "speedup_vs_driver": ms_driver / ms,
            "plan_and_autotune_s": plan_s,
            "launches_per_run": int(desc.strip().splitlines()[-1].split()[-1]),
            "stage_launches": {"ms_per_run": ms_stages, "launches_per_run": launches_stages,
                               "value": px / (ms_stages * 1e-3)}}


def leg_adjoint(torch, plink, synth, args):
    """Forward (coherence + linking with phases) and adjoint at 512x512, N=20."""
    wl = synth.WORKLOADS["adjoint"]
    z = synth.make_stack(wl, seed=args.seed, device="cuda")
    mean, var = plink.amplitude_stats(z)
    mask, _ = plink.shp_select(mean, var, wl.n_new, wl.window, wl.alpha)
    state = {}

    def fwd():
        coh = plink.estimate_coherence(z, mask, wl.window)
        state["r"] = plink.phase_link(coh, ref=0, want_phase=True)

    fwd()
    g = torch.randn((wl.N, wl.R * wl.C), device="cuda", generator=torch.Generator("cuda").manual_seed(1))
    ws = torch.empty((plink.phase_link_vjp_workspace(wl.N, wl.R, wl.C, wl.window),), dtype=torch.uint8,
                     device="cuda")
    flags = state["r"][2]
    ms_f = time_steps(torch, fwd, 10, 3)["median"]
    ms_b = time_steps(torch, lambda: plink.phase_link_vjp(z, mask, flags, wl.window, 0, g, workspace=ws), 10, 3)["median"]
    del ws
    ms_b64 = time_steps(torch, lambda: plink.phase_link_vjp(z, mask, flags, wl.window, 0, g, precision="fp64"),
                        3, 1)["median"]
    return {"workload": f"{wl.R}x{wl.C}, N={wl.N}, half-window {wl.window[0]}x{wl.window[1]}, stride 1",
            "forward_ms": ms_f, "vjp_ms": ms_b, "vjp_fp64_ms": ms_b64, "unit": "ms"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(this build runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.calibrate_copy:
        n = 1 << 28  # 2^28 float32 = 1 GiB each way
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": 4 * n, "calibrate_copy_bytes_written": 4 * n,
                          "launches": 3}))
        return

    import paper_2511_12051_amd as plink
    import synth
    plink.load()
    if args.only_sequence:
        print(json.dumps(leg_sequence(torch, plink, synth, args, args.precision)), flush=True)
        return
    wl = synth.WORKLOADS[args.workload]
    print(f"[bench] generating {wl.name} {wl.N}x{wl.R}x{wl.C} on cuda:0", file=sys.stderr, flush=True)
    stack = synth.make_stack(wl, seed=args.seed, device="cuda")
    torch.cuda.synchronize()
    oR, oC = wl.out_shape
    P = oR * oC

    results = {}
    precs = [args.precision] + ([] if args.no_compare else [p for p in ("bf16", "fp32") if p != args.precision])
    for prec in precs:
        results[prec] = measure(torch, plink, wl, stack, prec, args.steps, args.warmup, args.skip_fused)
    del stack
    torch.cuda.empty_cache()

    main_r = results[args.precision]
    alg, stage_roof = stage_rooflines(wl, main_r, args.precision)
    st = main_r["stages"]
    dom = max(st, key=st.get)
    roof = roofline(alg[dom], st[dom])
    roof["kernel"] = kernel_name(dom, wl, args.precision)
    roof["traffic"] = measured_traffic(roof["kernel"], wl, args.precision)
    roof["per_launch"] = {k: alg[dom][k] for k in ("bytes", "flops", "flops_fp64", "flops_fp32") if k in alg[dom]}
    roof["launch_ms"] = st[dom]
    if dom == "link":
        # the same flops against FP32 at the packed-instruction peak (157.3 TFLOP/s)
        t_ideal = alg[dom]["flops_fp64"] / 78.6e12 + alg[dom]["flops_fp32"] / 157.3e12
        roof["frac_with_packed_fp32_peak"] = t_ideal / (st[dom] * 1e-3)

    # the headline step is the fused one (coherence straight into linking
    # through bands of packed triangles, the full N x N C never written) when
    # it was timed; the split step (every stage its own call) is reported beside it
    fz = main_r["fused"]
    head_ms = fz["ms_per_step"] if fz else main_r["ms"]
    line = {
        "metric": "phase-linked pixels/sec at N=15/25 within 1e-3 rad of FP64 oracle; mixed vs FP32",
        "value": P / (head_ms * 1e-3),
        "unit": "pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head_ms,
        "step": "fused" if fz else "split",
        "split_ms_per_step": main_r["ms"],
        "split_ms_per_step_mean": main_r["ms_mean"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x2->f32" if args.precision == "bf16" else "f32",
        "data": "synthetic",
        "config": {"workload": describe(wl), "precision": args.precision},
        "stage_ms": {k: round(v, 4) for k, v in st.items()},
        "roofline": roof,
        "stage_roofline": stage_roof,
    }
    for prec, r in results.items():
        if prec != args.precision:
            line[f"{prec}_value"] = r["value"]
            line[f"{prec}_ms_per_step"] = r["ms"]
            line[f"{prec}_stage_ms"] = {k: round(v, 4) for k, v in r["stages"].items()}
    if "fp32" in results and "bf16" in results:
        line["mixed_speedup_vs_fp32"] = results["fp32"]["ms"] / results["bf16"]["ms"]
    line["fused_path"] = {p: r["fused"] for p, r in results.items()}
    line["evd_fraction"] = main_r["evd_frac"]
    line["link_counters"] = main_r["link_counters"]
    if not args.only_main and args.workload in ("scale", "burst"):
        other = "burst" if args.workload == "scale" else "scale"
        line[other] = leg_other(torch, plink, synth, args, other, args.steps, args.warmup)
        line["sequential_batched"] = leg_sequence(torch, plink, synth, args, args.precision)
        line["adjoint"] = leg_adjoint(torch, plink, synth, args)
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on a crop (host cores)", file=sys.stderr, flush=True)
        rec, cwl, cz, corc = cpu_baseline(args.workload, args.seed, args.cpu_workers)
        line["cpu_baseline"] = rec
        print("[bench] GPU error against the oracle on the same crop", file=sys.stderr, flush=True)
        line["accuracy_vs_oracle"] = accuracy_vs_oracle(torch, plink, cwl, cz, corc)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
