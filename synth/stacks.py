"""Seeded synthetic SLC stacks (inputs only; none of the estimation method).

Signal model: circular complex Gaussian scatterers (paper Sec. 2.1) whose
coherence decays exponentially with temporal baseline,
gamma(t) = (gamma0 - gamma_inf) exp(-t / tau) + gamma_inf (paper Sec. 2.3),
with a true phase made of an uplifting deformation bowl plus turbulent
atmosphere (paper Sec. 2.3).  Each pixel draws

    z_i = A * exp(j phi_i) * n_i,
    n_i = sqrt(g0 - ginf) x_i + sqrt(ginf) w + sqrt(1 - g0) e_i,

where x is a unit AR(1) process with coefficient exp(-1/tau) (so that
cov(x_i, x_k) = exp(-|i-k|/tau)), w is one CN(0,1) draw shared by all epochs
and e_i are independent CN(0,1) draws.  Then cov(n) is exactly the Gamma of
the model above with unit diagonal.

Land cover (per pixel): distributed scatterers (DS), persistent scatterers (PS,
gamma0 = gamma_inf = 0.98, amplitude 10) and, for the burst-scale workloads,
spatially contiguous water (gamma0 = 0.05, gamma_inf = 0, amplitude 0.2).  DS
amplitudes follow a smooth log-normal field so that the amplitude test has
real structure to find.

Everything is drawn with torch on the requested device from explicitly seeded
generators; the same seed on the same device type gives identical stacks.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import torch

WAVELENGTH_M = 0.055  # C-band, as in the workload descriptions
TAU_EPOCHS = 5.0      # decorrelation time in epochs


@dataclass(frozen=True)
class Workload:
    """One synthetic workload: grid, stack composition, window and model."""
    name: str
    R: int
    C: int
    n_new: int                 # real SLCs in the mini-stack
    n_comp: int                # compressed SLCs in front of them
    window: tuple              # (half_x, half_y, stride_x, stride_y)
    alpha: float = 1e-3
    model: str = "tiny"        # land-cover model: "tiny" (C1/C4) or "burst"
    bursts: int = 1
    ministacks: int = 1        # > 1: sequential workload of n_new-SLC mini-stacks
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.n_new + self.n_comp

    @property
    def out_shape(self):
        hx, hy, sx, sy = self.window
        return self.R // sy, self.C // sx


WORKLOADS = {
    # 64x64, N=10, half-window 5x5, stride 1, single mini-stack
    "tiny": Workload("tiny", 64, 64, 10, 0, (5, 5, 1, 1), model="tiny"),
    # burst-scale single mini-stack: 2048x8192, N=15, half 11x5, stride 6x3
    "burst": Workload("burst", 2048, 8192, 15, 0, (11, 5, 6, 3), model="burst"),
    # sequential batched: 4 bursts of 1024x4096, 8 mini-stacks of 15
    "sequential": Workload("sequential", 1024, 4096, 15, 0, (11, 5, 6, 3), model="burst",
                           bursts=4, ministacks=8),
    # differentiation: 512x512, N=20, half 7x7, stride 1
    "adjoint": Workload("adjoint", 512, 512, 20, 0, (7, 7, 1, 1), model="tiny"),
    # mixed precision at scale: 4096x16384, N=25 (10 compressed + 15 new)
    "scale": Workload("scale", 4096, 16384, 15, 10, (11, 5, 6, 3), model="burst"),
}


def _seed(*parts) -> int:
    h = hashlib.sha256(repr(parts).encode()).digest()
    return int.from_bytes(h[:8], "little") & ((1 << 63) - 1)


def _gen(device, *parts) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(_seed(*parts))
    return g


def _cn(shape, gen, device):
    """CN(0, 1) samples (complex64)."""
    re = torch.randn(shape, generator=gen, device=device, dtype=torch.float32)
    im = torch.randn(shape, generator=gen, device=device, dtype=torch.float32)
    return torch.complex(re, im) * (1.0 / math.sqrt(2.0))


def smooth_field(R, C, sigma, gen, device):
    """Unit-variance, zero-mean Gaussian-filtered white noise [R, C] (float32)."""
    w = torch.randn((R, C), generator=gen, device=device, dtype=torch.float32)
    fy = torch.fft.fftfreq(R, device=device).reshape(-1, 1)
    fx = torch.fft.rfftfreq(C, device=device).reshape(1, -1)
    H = torch.exp(-2.0 * (math.pi * sigma) ** 2 * (fy * fy + fx * fx))
    f = torch.fft.irfft2(torch.fft.rfft2(w) * H, s=(R, C))
    f = f - f.mean()
    return f / f.std().clamp_min(1e-30)


def land_cover(wl: Workload, seed, burst, device):
    """Per-pixel (amplitude, gamma0, gamma_inf, class) with class 0 DS, 1 PS, 2 water."""
    R, C = wl.R, wl.C
    g = _gen(device, "cover", wl.name, seed, burst)
    amp = torch.exp(0.5 * smooth_field(R, C, 8.0, g, device))
    cls = torch.zeros((R, C), dtype=torch.uint8, device=device)
    if wl.model == "tiny":
        g0 = torch.full((R, C), 0.8, device=device)
        ps = torch.rand((R, C), generator=g, device=device) < 0.10
    else:
        water_f = smooth_field(R, C, 24.0, g, device)
        thr = torch.quantile(water_f.flatten()[:: max(1, (R * C) // 1_000_000)].double(), 0.30)
        water = water_f < thr.float()
        ps = (~water) & (torch.rand((R, C), generator=g, device=device) < 2.0 / 7.0)
        gf = smooth_field(R, C, 16.0, g, device)
        # rank-map the smooth field to U(0.3, 0.9): use the normal CDF of a unit field
        g0 = 0.3 + 0.6 * 0.5 * (1.0 + torch.erf(gf / math.sqrt(2.0)))
        cls[water] = 2
        amp = torch.where(water, torch.full_like(amp, 0.2), amp)
        g0 = torch.where(water, torch.full_like(g0, 0.05), g0)
    cls[ps] = 1
    amp = torch.where(ps, torch.full_like(amp, 10.0), amp)
    g0 = torch.where(ps, torch.full_like(g0, 0.98), g0)
    ginf = torch.full_like(g0, 0.1)
    ginf = torch.where(ps, torch.full_like(ginf, 0.98), ginf)
    ginf = torch.where(cls == 2, torch.zeros_like(ginf), ginf)
    return amp, g0, ginf, cls


def true_phase(wl: Workload, seed, burst, epochs, device):
    """True phase of each epoch [len(epochs), R, C]: deformation bowl with a
    peak rate of 5 mm/epoch plus 1-rad turbulent atmosphere per epoch."""
    R, C = wl.R, wl.C
    yy = torch.arange(R, device=device, dtype=torch.float32).reshape(-1, 1) - (R - 1) / 2
    xx = torch.arange(C, device=device, dtype=torch.float32).reshape(1, -1) - (C - 1) / 2
    sb = min(R, C) / 6.0
    rate = 0.005 * torch.exp(-(yy * yy + xx * xx) / (2 * sb * sb))  # m / epoch
    out = torch.empty((len(epochs), R, C), device=device, dtype=torch.float32)
    for k, t in enumerate(epochs):
        ga = _gen(device, "atmo", wl.name, seed, burst, int(t))
        out[k] = 4 * math.pi / WAVELENGTH_M * rate * float(t) + smooth_field(R, C, 16.0, ga, device)
    return out


class _Noise:
    """Epoch-by-epoch generator of the correlated noise n_i of one burst."""

    def __init__(self, wl, seed, burst, g0, ginf, device):
        self.g = _gen(device, "noise", wl.name, seed, burst)
        self.device = device
        self.shape = g0.shape
        self.a = torch.sqrt((g0 - ginf).clamp_min(0))
        self.b = torch.sqrt(ginf)
        self.c = torch.sqrt((1 - g0).clamp_min(0))
        self.rho = math.exp(-1.0 / TAU_EPOCHS)
        self.w = _cn(self.shape, self.g, device)
        self.x = None

    def next(self):
        e = _cn(self.shape, self.g, self.device)
        u = _cn(self.shape, self.g, self.device)
        if self.x is None:
            self.x = u
        else:
            self.x = self.rho * self.x + math.sqrt(1 - self.rho ** 2) * u
        return self.a * self.x + self.b * self.w + self.c * e


def make_stack(wl: Workload | str, seed: int = 0, device="cpu", burst: int = 0,
               with_truth: bool = False):
    """Stack [n_comp + n_new, R, C] complex64 for a single-mini-stack workload.

    The n_comp compressed planes (if any) are built analytically: each one is
    the projection of 15 earlier epochs onto their true phases, i.e. the sum
    of their noise times the amplitude and exp(j phi_0) of the first new epoch
    (a compressed SLC inherits the reference phase)."""
    if isinstance(wl, str):
        wl = WORKLOADS[wl]
    device = torch.device(device)
    amp, g0, ginf, cls = land_cover(wl, seed, burst, device)
    noise = _Noise(wl, seed, burst, g0, ginf, device)
    block = 15
    n_hist = wl.n_comp * block
    first = n_hist
    phi = true_phase(wl, seed, burst, range(first, first + wl.n_new), device)
    out = torch.empty((wl.N, wl.R, wl.C), dtype=torch.complex64, device=device)
    ref = torch.polar(amp, phi[0])
    for b in range(wl.n_comp):
        acc = torch.zeros_like(out[0])
        for _ in range(block):
            acc += noise.next()
        out[b] = ref * acc
    for i in range(wl.n_new):
        out[wl.n_comp + i] = torch.polar(amp, phi[i]) * noise.next()
    if with_truth:
        return out, {"phase": phi, "amp": amp, "gamma0": g0, "gamma_inf": ginf, "cls": cls}
    return out


def make_sequence(wl: Workload | str, seed: int = 0, device="cpu", burst: int = 0,
                  ministacks: int | None = None, with_truth: bool = False):
    """All epochs of a sequential workload: [ministacks * n_new, R, C]."""
    if isinstance(wl, str):
        wl = WORKLOADS[wl]
    device = torch.device(device)
    K = wl.ministacks if ministacks is None else ministacks
    T = K * wl.n_new
    amp, g0, ginf, cls = land_cover(wl, seed, burst, device)
    noise = _Noise(wl, seed, burst, g0, ginf, device)
    phi = true_phase(wl, seed, burst, range(T), device)
    out = torch.empty((T, wl.R, wl.C), dtype=torch.complex64, device=device)
    for i in range(T):
        out[i] = torch.polar(amp, phi[i]) * noise.next()
    if with_truth:
        return out, {"phase": phi, "amp": amp, "gamma0": g0, "gamma_inf": ginf, "cls": cls}
    return out


def crop(wl: Workload | str, R: int, C: int, name_suffix="crop") -> Workload:
    """Same model and window on a smaller grid (oracle-sized parity cases)."""
    if isinstance(wl, str):
        wl = WORKLOADS[wl]
    return Workload(f"{wl.name}-{name_suffix}", R, C, wl.n_new, wl.n_comp, wl.window, wl.alpha,
                    wl.model, 1, wl.ministacks)
