#!/usr/bin/env python3
"""Throughput of the phase-linking hot path on one MI355X.

One step = amplitude statistics -> GLRT SHP masks -> sample coherence ->
EMI/EVD phase linking -> compressed SLC over one synthetic mini-stack that is
already resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload burst|scale|tiny]
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
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="burst")
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp32"])
    ap.add_argument("--no-compare", action="store_true", help="skip the other precision")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--only-main", action="store_true",
                    help="skip the N=25, batched-sequence and adjoint legs")
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


def time_steps(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def stage_times(torch, path, steps):
    """Average device time of each stage, HIP events on the stream the kernels use."""
    names = ["stats", "glrt", "coherence", "link", "compress"]
    acc = {n: 0.0 for n in names}
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
            acc[n] += ev[i].elapsed_time(ev[i + 1])
    return {n: v / steps for n, v in acc.items()}


def algorithmic(wl, shp_sum, P, prec):
    """Algorithmic bytes and flops of each stage (one launch each) and the
    peak each is measured against."""
    R, C, N, M = wl.R, wl.C, wl.N, wl.n_new
    nw = ((2 * wl.window[0] + 1) * (2 * wl.window[1] + 1) + 31) // 32
    px = R * C
    mfma_peak = PEAK["bf16_mfma_TFLOPs"] if prec == "bf16" else PEAK["fp32_mfma_TFLOPs"]
    return {
        "stats": {"bytes": px * M * 8 + px * 16},
        "glrt": {"bytes": px * 16 + P * nw * 4 + P * 2},
        # complex MACs over the N(N+1)/2 unique entries of each Hermitian A,
        # 8 flops each, over the pixel's SHPs
        "coherence": {"bytes": px * N * 8 + P * nw * 4 + P * N * N * 8,
                      "flops": shp_sum * (N * (N + 1) // 2) * 8, "flop_peak": mfma_peak,
                      "flop_bound": "mfma"},
        # EMI per pixel: one N x N FP64 inverse (2 N^3), one complex inverse
        # (8 N^3) and ten complex mat-vecs (8 N^2 each); vector ALU peak
        "link": {"bytes": P * N * N * 8 + P * N * 8 + P * 5,
                 "flops": P * (2 * N ** 3 + 8 * N ** 3 + 10 * 8 * N ** 2),
                 "flop_peak": PEAK["fp32_valu_TFLOPs"], "flop_bound": "alu"},
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


def cpu_baseline(wl_name, seed):
    """The FP64 oracle on a bounded crop of the same workload (host cores)."""
    import numpy as np

    import synth
    from oracle import plink_oracle as O
    wl = synth.crop(wl_name, 576 if wl_name != "tiny" else 64, 1536 if wl_name != "tiny" else 64)
    z = synth.make_stack(wl, seed=seed).numpy()
    t0, c0 = time.perf_counter(), time.process_time()
    r = O.link_ministack(z, wl.n_comp, wl.window, wl.alpha, max(0, wl.n_comp - 1))
    wall, cpu = time.perf_counter() - t0, time.process_time() - c0
    P = int(np.prod(wl.out_shape))
    return {"value": P / wall, "unit": "pixels/s", "cores": max(1, round(cpu / wall)),
            "kind": "oracle",
            "sample": f"{wl.R}x{wl.C} crop of the {wl_name} workload (N={wl.N}, window "
                      f"{wl.window}), {P} output pixels, {wall:.1f} s wall"}


def run_path(torch, plink, wl, stack, precs, steps, warmup):
    """ms/step, per-stage ms and solver counters of the single-call path."""
    out = {}
    oR, oC = wl.out_shape
    P = oR * oC
    for prec in precs:
        path = Path(plink, wl, stack, prec)
        ms = time_steps(torch, path.step, steps, warmup)
        stages = stage_times(torch, path, max(3, steps // 2))
        out[prec] = {"ms": ms, "stages": stages, "value": P / (ms * 1e-3)}
    return out


def leg_n25(torch, plink, synth, args):
    """Mixed precision at scale: 4096x16384, N=25 (10 compressed + 15 new)."""
    wl = synth.WORKLOADS["scale"]
    print(f"[bench] generating {wl.name} {wl.N}x{wl.R}x{wl.C}", file=sys.stderr, flush=True)
    stack = synth.make_stack(wl, seed=args.seed, device="cuda")
    r = run_path(torch, plink, wl, stack, ["bf16", "fp32"], 3, 1)
    del stack
    torch.cuda.empty_cache()
    return {"workload": f"{wl.R}x{wl.C}, N={wl.N} ({wl.n_comp} compressed + {wl.n_new} new), "
                        f"half-window {wl.window[0]}x{wl.window[1]}, stride {wl.window[2]}x{wl.window[3]}",
            "value": r["bf16"]["value"], "unit": "pixels/s", "ms_per_step": r["bf16"]["ms"],
            "stage_ms": {k: round(v, 4) for k, v in r["bf16"]["stages"].items()},
            "fp32_value": r["fp32"]["value"], "fp32_ms_per_step": r["fp32"]["ms"],
            "fp32_stage_ms": {k: round(v, 4) for k, v in r["fp32"]["stages"].items()},
            "mixed_speedup_vs_fp32": r["fp32"]["ms"] / r["bf16"]["ms"]}


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
    batch.run()  # captures the graph
    ms = time_steps(torch, batch.run, 3, 1)
    desc = batch.describe()

    def driver():
        for z in seqs:
            s = plink.Sequential(wl.R, wl.C, M, Kmax, wl.window, wl.alpha, precision=prec)
            for k in range(n):
                s.push(z[k * M:(k + 1) * M])
            s.close()

    ms_driver = time_steps(torch, driver, 2, 1)
    batch.close()
    px = wl.bursts * n * oR * oC
    return {"workload": f"{wl.bursts} bursts x {n} mini-stacks of {M} SLCs, {wl.R}x{wl.C}, N=15..22, "
                        f"half-window {wl.window[0]}x{wl.window[1]}, stride {wl.window[2]}x{wl.window[3]}",
            "precision": prec, "value": px / (ms * 1e-3), "unit": "pixels/s", "ms_per_run": ms,
            "output_pixels": px, "driver_ms": ms_driver, "speedup_vs_driver": ms_driver / ms,
            "plan_and_autotune_s": plan_s,
            "launches_per_run": int(desc.strip().splitlines()[-1].split()[-1])}


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
    ms_f = time_steps(torch, fwd, 5, 1)
    ms_b = time_steps(torch, lambda: plink.phase_link_vjp(z, mask, flags, wl.window, 0, g, workspace=ws), 5, 1)
    return {"workload": f"{wl.R}x{wl.C}, N={wl.N}, half-window {wl.window[0]}x{wl.window[1]}, stride 1",
            "forward_ms": ms_f, "vjp_ms": ms_b, "unit": "ms"}


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
    wl = synth.WORKLOADS[args.workload]
    print(f"[bench] generating {wl.name} {wl.N}x{wl.R}x{wl.C} on cuda:0", file=sys.stderr, flush=True)
    stack = synth.make_stack(wl, seed=args.seed, device="cuda")
    torch.cuda.synchronize()
    oR, oC = wl.out_shape
    P = oR * oC

    results = {}
    precs = [args.precision] + ([] if args.no_compare else [p for p in ("bf16", "fp32") if p != args.precision])
    for prec in precs:
        path = Path(plink, wl, stack, prec)
        print(f"[bench] {prec}: warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
        ms = time_steps(torch, path.step, args.steps, args.warmup)
        stages = stage_times(torch, path, max(3, args.steps // 2))
        m, coh, ln, k = path.step()
        cnt = plink.new_counters()
        plink.phase_link(coh, ref=path.ref, counters=cnt)
        torch.cuda.synchronize()
        cnt = dict(zip(plink.COUNTERS, cnt.cpu().tolist()))
        shp_sum = int(m[1].to(torch.int32).sum().item())
        flags = ln[2].cpu().numpy()
        results[prec] = {"ms": ms, "stages": stages, "shp_sum": shp_sum,
                         "evd_frac": float(np.mean(flags == 1)), "invalid_frac": float(np.mean(flags == 2)),
                         "link_counters": {"iters_per_pixel": cnt["iters"] / P,
                                           "shift_retries_per_pixel": cnt["shift_retry"] / P,
                                           "not_converged": cnt["not_converged"]}}
        print(f"[bench] {prec}: {ms:.3f} ms/step, stages {json.dumps({k: round(v, 4) for k, v in stages.items()})}",
              file=sys.stderr, flush=True)

    main_r = results[args.precision]
    alg = algorithmic(wl, main_r["shp_sum"], P, args.precision)
    st = main_r["stages"]
    dom = max(st, key=st.get)
    roof = roofline(alg[dom], st[dom])
    roof["kernel"] = kernel_name(dom, wl, args.precision)
    roof["traffic"] = measured_traffic(roof["kernel"], wl, args.precision)
    stage_roof = {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv)
                      for kk, vv in roofline(alg[k], st[k]).items()} for k in st}

    line = {
        "metric": "phase-linked pixels/sec at N=15/25 within 1e-3 rad of FP64 oracle; mixed vs FP32",
        "value": P / (main_r["ms"] * 1e-3),
        "unit": "pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_r["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x2->f32" if args.precision == "bf16" else "f32",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.R}x{wl.C} grid, N={wl.N} ({wl.n_comp} compressed + "
                               f"{wl.n_new} new), half-window {wl.window[0]}x{wl.window[1]}, "
                               f"stride {wl.window[2]}x{wl.window[3]}, {P} output pixels",
                   "precision": args.precision},
        "stage_ms": {k: round(v, 4) for k, v in st.items()},
        "roofline": roof,
        "stage_roofline": stage_roof,
    }
    for prec, r in results.items():
        if prec != args.precision:
            line[f"{prec}_value"] = P / (r["ms"] * 1e-3)
            line[f"{prec}_ms_per_step"] = r["ms"]
            line[f"{prec}_stage_ms"] = {k: round(v, 4) for k, v in r["stages"].items()}
            line["mixed_speedup_vs_fp32"] = (results["fp32"]["ms"] / results["bf16"]["ms"]
                                             if "fp32" in results and "bf16" in results else None)
    line["evd_fraction"] = main_r["evd_frac"]
    line["link_counters"] = main_r["link_counters"]
    if not args.only_main and args.workload == "burst":
        line["n25"] = leg_n25(torch, plink, synth, args)
        line["sequential_batched"] = leg_sequence(torch, plink, synth, args, args.precision)
        line["adjoint"] = leg_adjoint(torch, plink, synth, args)
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on a crop (host cores)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(args.workload, args.seed)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
