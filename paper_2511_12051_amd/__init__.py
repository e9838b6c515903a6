"""Python binding of libplink (MI355X / gfx950 sequential phase linking).

Argument marshalling only: every step runs in the library's HIP kernels on the
tensors' device, enqueued on torch's current stream.  There is no CPU path:
if the shared library is missing or no GPU is present the calls raise.

Method: Staniewicz et al., arXiv 2511.12051 (sequential EMI phase linking
with compressed SLCs).  The C declarations, with the passages they follow,
are in include/plink.h.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

__all__ = [
    "PlinkError", "load", "library_path", "output_grid", "mask_words", "amplitude_stats",
    "merge_amplitude_stats", "shp_select", "estimate_coherence", "phase_link",
    "compress_ministack", "Sequential", "new_counters", "phase_link_vjp", "phase_link_vjp_workspace",
    "phase_link_fused", "phase_link_fused_workspace", "sync_report", "ps_regrid", "phase_similarity",
    "network_size", "network_invert_l1",
    "PhaseLink", "Batch", "COUNTERS", "FLAG_EMI", "FLAG_EVD",
    "FLAG_INVALID", "MAX_N",
]

MAX_N = 32
FLAG_EMI, FLAG_EVD, FLAG_INVALID = 0, 1, 2
#: names of the counters array entries (index = position); entries 8..23 are
#: the histogram of eigenvector iterations per pixel (see sync_report)
COUNTERS = ("glrt_band", "glrt_recheck", "evd", "invalid", "not_converged", "shift_retry", "iters")
NUM_COUNTERS = 24
ITER_HIST = 8
_PREC = {"fp32": 0, "bf16": 1, "split_bf16": 1}
_METHOD = {"emi": 0, "evd": 1}

_HERE = os.path.dirname(os.path.abspath(__file__))


def library_path() -> str:
    return os.environ.get("PLINK_LIBRARY", os.path.join(_HERE, "libplink.so"))


class PlinkError(RuntimeError):
    pass


class _Window(ctypes.Structure):
    _fields_ = [("half_x", ctypes.c_int32), ("half_y", ctypes.c_int32),
                ("stride_x", ctypes.c_int32), ("stride_y", ctypes.c_int32)]


class _SeqParams(ctypes.Structure):
    _fields_ = [("R", ctypes.c_int64), ("C", ctypes.c_int64), ("M", ctypes.c_int32),
                ("K_max", ctypes.c_int32), ("w", _Window), ("alpha", ctypes.c_double),
                ("precision", ctypes.c_int32), ("method", ctypes.c_int32),
                ("reference", ctypes.c_int32), ("weight_decay", ctypes.c_double)]

    def __init__(self, R=0, C=0, M=0, K_max=0, w=None, alpha=1e-3, precision=0, method=0, reference=0,
                 weight_decay=1.0):
        super().__init__(R, C, M, K_max, w if w is not None else _Window(0, 0, 1, 1), alpha, precision, method,
                         reference, weight_decay)


class _Report(ctypes.Structure):
    _fields_ = [("glrt_band", ctypes.c_int64), ("glrt_recheck", ctypes.c_int64),
                ("evd_fallbacks", ctypes.c_int64), ("invalid", ctypes.c_int64),
                ("not_converged", ctypes.c_int64), ("shift_retries", ctypes.c_int64),
                ("iterations", ctypes.c_int64), ("iter_hist", ctypes.c_int64 * 16)]


class _BatchItem(ctypes.Structure):
    _fields_ = [("stack", ctypes.c_void_p), ("R", ctypes.c_int64), ("C", ctypes.c_int64),
                ("N", ctypes.c_int32), ("first_real", ctypes.c_int32), ("ref_idx", ctypes.c_int32),
                ("mean", ctypes.c_void_p), ("var", ctypes.c_void_p), ("n_eff", ctypes.c_double),
                ("phasors", ctypes.c_void_p), ("flags", ctypes.c_void_p), ("kappa", ctypes.c_void_p),
                ("planes", ctypes.POINTER(ctypes.c_void_p)), ("level", ctypes.c_int32)]


_lib = None
_P = ctypes.c_void_p
_I32, _I64, _D = ctypes.c_int32, ctypes.c_int64, ctypes.c_double

_SIGNATURES = {
    "pl_version": (ctypes.c_char_p, []),
    "pl_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "pl_last_error": (ctypes.c_char_p, []),
    "pl_output_grid": (ctypes.c_int, [_I64, _I64, _Window, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "pl_mask_words": (_I32, [_Window]),
    "pl_amplitude_stats": (ctypes.c_int, [_P, _I32, _I64, _I64, _P, _P, _P]),
    "pl_merge_amplitude_stats": (ctypes.c_int, [_P, _P, ctypes.POINTER(_D), _I32, _I64, _I64, _P, _P, _P]),
    "pl_shp_select": (ctypes.c_int, [_P, _P, _I64, _I64, _D, _Window, _D, _P, _P, _P, _P]),
    "pl_estimate_coherence": (ctypes.c_int, [_P, _I32, _I64, _I64, _Window, _P, ctypes.c_int, _P, _P]),
    "pl_phase_link": (ctypes.c_int, [_P, _I32, _I64, _I32, ctypes.c_int, _P, _P, _P, _P, _P, _P, _P]),
    "pl_sync_report": (ctypes.c_int, [_P, _P, ctypes.POINTER(_Report)]),
    "pl_phase_link_fused_workspace": (ctypes.c_int, [_I32, _I64, _I64, _Window, ctypes.POINTER(ctypes.c_size_t),
                                                     ctypes.POINTER(ctypes.c_size_t)]),
    "pl_phase_link_fused": (ctypes.c_int, [_P, _I32, _I64, _I64, _Window, _P, ctypes.c_int, _I32, ctypes.c_int,
                                           _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "pl_phase_link_fused_noalloc": (ctypes.c_int, [_P, _I32, _I64, _I64, _Window, _P, ctypes.c_int, _I32,
                                                   ctypes.c_int, _P, _P, _P, _P, _P, _P, _P]),
    "pl_ps_regrid": (ctypes.c_int, [_P, _I32, _I64, _I64, _Window, _I32, _P, _P, _D, _P, _P, _P, _P, _P]),
    "pl_phase_similarity": (ctypes.c_int, [_P, _I32, _I64, _I64, _P, _I32, _I32, _P, _P]),
    "pl_network_size": (ctypes.c_int, [_I32, _I32, ctypes.POINTER(_I32)]),
    "pl_network_invert_l1": (ctypes.c_int, [_P, _I32, _I32, _I64, _D, _I32, _P, _P, _P]),
    "pl_phase_link_vjp_workspace": (ctypes.c_int, [_I32, _I64, _I64, _Window, ctypes.POINTER(ctypes.c_size_t)]),
    "pl_phase_link_vjp": (ctypes.c_int, [_P, _I32, _I64, _I64, _Window, _P, _P, _I32, ctypes.c_int, _P, _P,
                                         _P, ctypes.c_size_t, _P]),
    "pl_phase_link_vjp64_workspace": (ctypes.c_int, [_I32, _I64, _I64, _Window, ctypes.POINTER(ctypes.c_size_t)]),
    "pl_phase_link_vjp64": (ctypes.c_int, [_P, _I32, _I64, _I64, _Window, _P, _P, _I32, _P, _P, _P,
                                           ctypes.c_size_t, _P]),
    "pl_compress_ministack": (ctypes.c_int, [_P, _I32, _I32, _I64, _I64, _Window, _P, _P, _P]),
    "pl_batch_plan": (ctypes.c_int, [ctypes.POINTER(_BatchItem), _I32, _Window, _D, ctypes.c_int, ctypes.c_int,
                                     _I32, _P, ctypes.POINTER(_P)]),
    "pl_batch_run": (ctypes.c_int, [_P, _P]),
    "pl_batch_destroy": (ctypes.c_int, [_P]),
    "pl_batch_describe": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.c_size_t]),
    "pl_batch_set_single_launch": (ctypes.c_int, [_P, ctypes.c_int32]),
    "pl_batch_check": (ctypes.c_int, [_P, ctypes.c_void_p]),
    "pl_batch_set_wait_limit": (ctypes.c_int, [_P, ctypes.c_uint32]),
    "pl_seq_create": (ctypes.c_int, [ctypes.POINTER(_SeqParams), ctypes.POINTER(_P)]),
    "pl_seq_workspace_size": (ctypes.c_int, [ctypes.POINTER(_SeqParams), ctypes.POINTER(ctypes.c_size_t)]),
    "pl_seq_create_in": (ctypes.c_int, [ctypes.POINTER(_SeqParams), ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.POINTER(_P)]),
    "pl_seq_destroy": (ctypes.c_int, [_P]),
    "pl_seq_count": (ctypes.c_int, [_P, ctypes.POINTER(_I64)]),
    "pl_seq_push": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "pl_seq_state_size": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "pl_seq_last_mask": (ctypes.c_int, [_P, _P, _P]),
    "pl_seq_save": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P]),
    "pl_seq_load": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P]),
}


def load():
    """Loads libplink.so (after torch, so both use torch's HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise PlinkError(f"{path} not built: run python -m paper_2511_12051_amd.build")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, what: str):
    if status != 0:
        lib = load()
        msg = lib.pl_last_error().decode()
        raise PlinkError(f"{what}: {lib.pl_status_string(status).decode()}: {msg}")


def _win(window) -> _Window:
    hx, hy, sx, sy = (int(v) for v in window)
    return _Window(hx, hy, sx, sy)


def _stream(t: torch.Tensor):
    if t.device.type != "cuda":
        raise PlinkError("tensors must live on a GPU (no CPU path)")
    return _P(torch.cuda.current_stream(t.device).cuda_stream)


def _ptr(t):
    return None if t is None else _P(t.data_ptr())


def _need(t: torch.Tensor, dtype, ndim, name):
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or t.dim() != ndim:
        raise PlinkError(f"{name}: expected a {ndim}-d {dtype} tensor")
    if not t.is_contiguous():
        raise PlinkError(f"{name}: tensor must be contiguous")
    if t.device.type != "cuda":
        raise PlinkError(f"{name}: tensor must live on a GPU (no CPU path)")


def output_grid(R: int, C: int, window):
    lib = load()
    oR, oC = _I64(), _I64()
    _check(lib.pl_output_grid(int(R), int(C), _win(window), ctypes.byref(oR), ctypes.byref(oC)),
           "output_grid")
    return oR.value, oC.value


def mask_words(window) -> int:
    n = load().pl_mask_words(_win(window))
    if n <= 0:
        raise PlinkError("mask_words: invalid window")
    return n


def new_counters(device="cuda"):
    """Zeroed device counter array (see COUNTERS for the entries)."""
    return torch.zeros(NUM_COUNTERS, dtype=torch.int64, device=device)


def sync_report(counters: torch.Tensor) -> dict:
    """Waits for the current stream and returns the counters as a dict, with
    the iteration histogram under "iter_hist" (entry 15: 15 or more)."""
    if counters.dtype != torch.int64 or counters.numel() < NUM_COUNTERS or not counters.is_contiguous():
        raise PlinkError("sync_report: expected a contiguous int64 counters tensor")
    rep = _Report()
    _check(load().pl_sync_report(_stream(counters), _ptr(counters), ctypes.byref(rep)), "sync_report")
    out = {k: getattr(rep, k) for k, _ in _Report._fields_ if k != "iter_hist"}
    out["iter_hist"] = list(rep.iter_hist)
    return out


def amplitude_stats(slc: torch.Tensor):
    """Mean and population variance of |z| over images: [M,R,C] -> 2 x [R,C] float64."""
    _need(slc, torch.complex64, 3, "amplitude_stats")
    M, R, C = slc.shape
    mean = torch.empty((R, C), dtype=torch.float64, device=slc.device)
    var = torch.empty_like(mean)
    _check(load().pl_amplitude_stats(_ptr(slc), M, R, C, _ptr(mean), _ptr(var), _stream(slc)),
           "amplitude_stats")
    return mean, var


def merge_amplitude_stats(means: torch.Tensor, variances: torch.Tensor, weights):
    """Pooled statistics of G groups: [G,R,C] x 2 + G weights -> 2 x [R,C]."""
    _need(means, torch.float64, 3, "merge_amplitude_stats")
    _need(variances, torch.float64, 3, "merge_amplitude_stats")
    G, R, C = means.shape
    w = (_D * G)(*[float(x) for x in weights])
    mean = torch.empty((R, C), dtype=torch.float64, device=means.device)
    var = torch.empty_like(mean)
    _check(load().pl_merge_amplitude_stats(_ptr(means), _ptr(variances), w, G, R, C, _ptr(mean),
                                           _ptr(var), _stream(means)), "merge_amplitude_stats")
    return mean, var


def shp_select(mean: torch.Tensor, var: torch.Tensor, n_eff: float, window, alpha: float,
               counters: torch.Tensor | None = None):
    """GLRT SHP masks: -> (mask int32 [oR,oC,nwords] holding uint32 bits, count int16 [oR,oC])."""
    _need(mean, torch.float64, 2, "shp_select")
    _need(var, torch.float64, 2, "shp_select")
    R, C = mean.shape
    oR, oC = output_grid(R, C, window)
    nw = mask_words(window)
    mask = torch.empty((oR, oC, nw), dtype=torch.int32, device=mean.device)
    count = torch.empty((oR, oC), dtype=torch.int16, device=mean.device)
    _check(load().pl_shp_select(_ptr(mean), _ptr(var), R, C, float(n_eff), _win(window),
                                float(alpha), _ptr(mask), _ptr(count), _ptr(counters),
                                _stream(mean)), "shp_select")
    return mask, count


def estimate_coherence(stack: torch.Tensor, mask: torch.Tensor, window, precision="fp32"):
    """Normalised sample coherence over SHPs: -> complex64 [oR*oC, N, N]."""
    _need(stack, torch.complex64, 3, "estimate_coherence")
    _need(mask, torch.int32, 3, "estimate_coherence mask")
    N, R, C = stack.shape
    oR, oC = output_grid(R, C, window)
    if tuple(mask.shape) != (oR, oC, mask_words(window)):
        raise PlinkError("estimate_coherence: mask shape does not match the window")
    coh = torch.empty((oR * oC, N, N), dtype=torch.complex64, device=stack.device)
    _check(load().pl_estimate_coherence(_ptr(stack), N, R, C, _win(window), _ptr(mask),
                                        _PREC[precision], _ptr(coh), _stream(stack)),
           "estimate_coherence")
    return coh


def phase_link(coh: torch.Tensor, ref: int = 0, method="emi", counters=None, want_phase=False,
               want_tcoh=False):
    """EMI (EVD fallback) linked phasors: [P,N,N] -> (phasors [N,P], lambda [P], flags uint8 [P]),
    followed by the phases [N,P] (float32, radians) when want_phase and the
    temporal coherence [P] (float32) when want_tcoh."""
    _need(coh, torch.complex64, 3, "phase_link")
    P, N, N2 = coh.shape
    if N != N2:
        raise PlinkError("phase_link: matrices must be square")
    ph = torch.empty((N, P), dtype=torch.complex64, device=coh.device)
    phase = torch.empty((N, P), dtype=torch.float32, device=coh.device) if want_phase else None
    tcoh = torch.empty((P,), dtype=torch.float32, device=coh.device) if want_tcoh else None
    lam = torch.empty((P,), dtype=torch.float32, device=coh.device)
    flags = torch.empty((P,), dtype=torch.uint8, device=coh.device)
    _check(load().pl_phase_link(_ptr(coh), N, P, int(ref), _METHOD[method], _ptr(ph), _ptr(phase),
                                _ptr(lam), _ptr(tcoh), _ptr(flags), _ptr(counters), _stream(coh)), "phase_link")
    out = (ph, lam, flags)
    if want_phase:
        out += (phase,)
    if want_tcoh:
        out += (tcoh,)
    return out


def phase_link_fused_workspace(N: int, R: int, C: int, window):
    """(bytes of one output row, bytes of all rows) of packed coherence."""
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    _check(load().pl_phase_link_fused_workspace(int(N), int(R), int(C), _win(window), ctypes.byref(a),
                                                ctypes.byref(b)), "phase_link_fused_workspace")
    return a.value, b.value


def phase_link_fused(stack: torch.Tensor, mask: torch.Tensor, window, ref: int = 0, precision="fp32",
                     method="emi", counters=None, workspace: torch.Tensor | None = None,
                     want_phase=False, want_tcoh=False):
    """Coherence straight into phase linking, band by band through
    `workspace` (uint8 device tensor; default: every output row at once).
    Returns (phasors [N, oR*oC], lambda, flags[, phase][, tcoh]) like
    phase_link."""
    _need(stack, torch.complex64, 3, "phase_link_fused")
    _need(mask, torch.int32, 3, "phase_link_fused mask")
    N, R, C = stack.shape
    oR, oC = output_grid(R, C, window)
    if tuple(mask.shape) != (oR, oC, mask_words(window)):
        raise PlinkError("phase_link_fused: mask shape does not match the window")
    if workspace is None:
        workspace = torch.empty((phase_link_fused_workspace(N, R, C, window)[1],), dtype=torch.uint8,
                                device=stack.device)
    P = oR * oC
    dev = stack.device
    ph = torch.empty((N, P), dtype=torch.complex64, device=dev)
    phase = torch.empty((N, P), dtype=torch.float32, device=dev) if want_phase else None
    tcoh = torch.empty((P,), dtype=torch.float32, device=dev) if want_tcoh else None
    lam = torch.empty((P,), dtype=torch.float32, device=dev)
    flags = torch.empty((P,), dtype=torch.uint8, device=dev)
    _check(load().pl_phase_link_fused(_ptr(stack), N, R, C, _win(window), _ptr(mask), _PREC[precision], int(ref),
                                      _METHOD[method], _ptr(ph), _ptr(phase), _ptr(lam), _ptr(tcoh), _ptr(flags),
                                      _ptr(counters), _ptr(workspace),
                                      workspace.numel() * workspace.element_size(), _stream(stack)),
           "phase_link_fused")
    out = (ph, lam, flags)
    if want_phase:
        out += (phase,)
    if want_tcoh:
        out += (tcoh,)
    return out


def ps_regrid(stack: torch.Tensor, ref: int, window, mean: torch.Tensor, var: torch.Tensor,
              ds_phasors: torch.Tensor, threshold: float = 0.2, inplace=False):
    """PS selection (D_A <= threshold) and PS/DS regridding: -> (phasors
    [N, oR*oC], PS source index int64 [oR*oC] (-1: DS), PS mask uint8 [R,C])."""
    _need(stack, torch.complex64, 3, "ps_regrid")
    _need(mean, torch.float64, 2, "ps_regrid mean")
    _need(var, torch.float64, 2, "ps_regrid var")
    N, R, C = stack.shape
    oR, oC = output_grid(R, C, window)
    if ds_phasors.dtype != torch.complex64 or ds_phasors.numel() != N * oR * oC or not ds_phasors.is_contiguous():
        raise PlinkError("ps_regrid: ds_phasors must be contiguous complex64 [N, oR*oC]")
    out = ds_phasors if inplace else torch.empty((N, oR * oC), dtype=torch.complex64, device=stack.device)
    src = torch.empty((oR * oC,), dtype=torch.int64, device=stack.device)
    ps = torch.empty((R, C), dtype=torch.uint8, device=stack.device)
    _check(load().pl_ps_regrid(_ptr(stack), N, R, C, _win(window), int(ref), _ptr(mean), _ptr(var), float(threshold),
                               _ptr(ds_phasors), _ptr(out), _ptr(src), _ptr(ps), _stream(stack)), "ps_regrid")
    return out, src, ps


def phase_similarity(phasors: torch.Tensor, out_shape, radius: int, k: int = 3, flags=None):
    """gamma_s [oR*oC] (float32) of linked phasors [N, oR*oC]."""
    oR, oC = out_shape
    if phasors.dtype != torch.complex64 or phasors.dim() != 2 or phasors.shape[1] != oR * oC \
            or not phasors.is_contiguous():
        raise PlinkError("phase_similarity: phasors must be contiguous complex64 [N, oR*oC]")
    if flags is not None and (flags.dtype != torch.uint8 or flags.numel() != oR * oC or not flags.is_contiguous()):
        raise PlinkError("phase_similarity: flags must be contiguous uint8 [oR*oC]")
    out = torch.empty((oR * oC,), dtype=torch.float32, device=phasors.device)
    _check(load().pl_phase_similarity(_ptr(phasors), phasors.shape[0], oR, oC, _ptr(flags), int(radius), int(k),
                                      _ptr(out), _stream(phasors)), "phase_similarity")
    return out


def network_size(N: int, k: int = 3) -> int:
    n = _I32()
    _check(load().pl_network_size(int(N), int(k), ctypes.byref(n)), "network_size")
    return n.value


def network_invert_l1(ifg: torch.Tensor, N: int, k: int = 3, rho: float = 1.0, iters: int = 200):
    """L1 inversion of unwrapped interferograms [n_ifg, P] (float32) of the
    nearest-k network: -> (x [N-1, P], residual ||Ax - b||_1 [P])."""
    _need(ifg, torch.float32, 2, "network_invert_l1")
    if ifg.shape[0] != network_size(N, k):
        raise PlinkError("network_invert_l1: ifg rows do not match the network")
    P = ifg.shape[1]
    x = torch.empty((N - 1, P), dtype=torch.float32, device=ifg.device)
    res = torch.empty((P,), dtype=torch.float32, device=ifg.device)
    _check(load().pl_network_invert_l1(_ptr(ifg), int(N), int(k), P, float(rho), int(iters), _ptr(x), _ptr(res),
                                       _stream(ifg)), "network_invert_l1")
    return x, res


def phase_link_vjp_workspace(N: int, R: int, C: int, window) -> int:
    """Bytes of device workspace that phase_link_vjp needs."""
    n = ctypes.c_size_t()
    _check(load().pl_phase_link_vjp_workspace(int(N), int(R), int(C), _win(window), ctypes.byref(n)),
           "phase_link_vjp_workspace")
    return n.value


def phase_link_vjp(stack: torch.Tensor, mask: torch.Tensor, flags: torch.Tensor, window, ref: int,
                   grad_phase: torch.Tensor, precision="fp32", workspace: torch.Tensor | None = None):
    """dL/dz (as dL/dRe + j dL/dIm, complex64 [N,R,C]) of the linked phases given
    dL/dphi (float32 [N, oR*oC] or [N,oR,oC]); mask and EMI/EVD flags held fixed.
    precision "fp64" runs every step of the adjoint in double precision."""
    if precision == "fp64":
        return _phase_link_vjp64(stack, mask, flags, window, ref, grad_phase, workspace)
    _need(stack, torch.complex64, 3, "phase_link_vjp")
    _need(mask, torch.int32, 3, "phase_link_vjp mask")
    N, R, C = stack.shape
    oR, oC = output_grid(R, C, window)
    if tuple(mask.shape) != (oR, oC, mask_words(window)):
        raise PlinkError("phase_link_vjp: mask shape does not match the window")
    if flags.dtype != torch.uint8 or flags.numel() != oR * oC or not flags.is_contiguous():
        raise PlinkError("phase_link_vjp: flags must be contiguous uint8 [oR*oC]")
    if (grad_phase.dtype != torch.float32 or grad_phase.numel() != N * oR * oC
            or not grad_phase.is_contiguous() or grad_phase.device != stack.device):
        raise PlinkError("phase_link_vjp: grad_phase must be contiguous float32 [N, oR*oC] on the stack's GPU")
    need = phase_link_vjp_workspace(N, R, C, window)
    if workspace is None:
        workspace = torch.empty((need,), dtype=torch.uint8, device=stack.device)
    grad = torch.empty_like(stack)
    _check(load().pl_phase_link_vjp(_ptr(stack), N, R, C, _win(window), _ptr(mask), _ptr(flags), int(ref),
                                    _PREC[precision], _ptr(grad_phase), _ptr(grad), _ptr(workspace),
                                    workspace.numel() * workspace.element_size(), _stream(stack)),
           "phase_link_vjp")
    return grad


def _phase_link_vjp64(stack, mask, flags, window, ref, grad_phase, workspace=None):
    _need(stack, torch.complex64, 3, "phase_link_vjp")
    _need(mask, torch.int32, 3, "phase_link_vjp mask")
    N, R, C = stack.shape
    oR, oC = output_grid(R, C, window)
    if tuple(mask.shape) != (oR, oC, mask_words(window)):
        raise PlinkError("phase_link_vjp: mask shape does not match the window")
    if flags.dtype != torch.uint8 or flags.numel() != oR * oC or not flags.is_contiguous():
        raise PlinkError("phase_link_vjp: flags must be contiguous uint8 [oR*oC]")
    if (grad_phase.dtype != torch.float32 or grad_phase.numel() != N * oR * oC
            or not grad_phase.is_contiguous() or grad_phase.device != stack.device):
        raise PlinkError("phase_link_vjp: grad_phase must be contiguous float32 [N, oR*oC] on the stack's GPU")
    n = ctypes.c_size_t()
    _check(load().pl_phase_link_vjp64_workspace(N, R, C, _win(window), ctypes.byref(n)), "phase_link_vjp64_workspace")
    if workspace is None or workspace.numel() * workspace.element_size() < n.value:
        workspace = torch.empty((n.value,), dtype=torch.uint8, device=stack.device)
    grad = torch.empty_like(stack)
    _check(load().pl_phase_link_vjp64(_ptr(stack), N, R, C, _win(window), _ptr(mask), _ptr(flags), int(ref),
                                      _ptr(grad_phase), _ptr(grad), _ptr(workspace),
                                      workspace.numel() * workspace.element_size(), _stream(stack)), "phase_link_vjp64")
    return grad


class PhaseLink(torch.autograd.Function):
    """Linked phases [N, oR, oC] of a stack [N, R, C] (complex64) for a fixed SHP
    mask, differentiable with respect to the stack (backward_precision "fp64"
    selects the FP64 adjoint; default: the forward's precision).  The forward is the fused
    coherence + linking entry point (no full-size coherence array); the
    backward recomputes the coherence and the eigen-solve inside the adjoint
    kernels (only the stack, the mask and the per-pixel EMI/EVD flags are
    kept)."""

    @staticmethod
    def forward(ctx, stack, mask, window, ref=0, precision="fp32", method="emi", backward_precision=None):
        N, R, C = stack.shape
        oR, oC = output_grid(R, C, window)
        _, _, flags, phase = phase_link_fused(stack, mask, window, ref, precision, method, want_phase=True)
        ctx.save_for_backward(stack, mask, flags)
        ctx.window, ctx.ref = tuple(window), int(ref)
        ctx.precision = backward_precision or precision
        ctx.mark_non_differentiable(flags)
        return phase.view(N, oR, oC), flags

    @staticmethod
    def backward(ctx, grad_phase, grad_flags=None):
        stack, mask, flags = ctx.saved_tensors
        g = grad_phase.to(torch.float32).contiguous()
        grad = phase_link_vjp(stack, mask, flags, ctx.window, ctx.ref, g, ctx.precision)
        return grad, None, None, None, None, None, None


def compress_ministack(stack: torch.Tensor, first_real: int, window, phasors: torch.Tensor):
    """Compressed SLC: stack [N,R,C], phasors [N,oR,oC] -> kappa complex64 [R,C]."""
    _need(stack, torch.complex64, 3, "compress_ministack")
    N, R, C = stack.shape
    oR, oC = output_grid(R, C, window)
    if phasors.dtype != torch.complex64 or phasors.numel() != N * oR * oC or not phasors.is_contiguous():
        raise PlinkError("compress_ministack: phasors must be contiguous complex64 [N,oR,oC]")
    kappa = torch.empty((R, C), dtype=torch.complex64, device=stack.device)
    _check(load().pl_compress_ministack(_ptr(stack), N, int(first_real), R, C, _win(window),
                                        _ptr(phasors), _ptr(kappa), _stream(stack)),
           "compress_ministack")
    return kappa


class Batch:
    """Independent mini-stacks run together: one persistent launch per stage
    and kernel variant, captured into a HIP graph on the first run and
    replayed afterwards.  Each item is a dict with either ``stack``
    (complex64 [N,R,C], compressed planes first) or ``planes`` (a list of N
    complex64 [R,C] tensors, e.g. compressed SLCs written by lower levels),
    and optional ``first_real`` (0), ``ref`` (0), ``mean``/``var`` (float64
    [R,C] statistics for the GLRT; computed from the real images when
    absent), ``n_eff``, ``level`` (0; levels run in increasing order),
    ``phasors`` (output tensor [N,oR,oC] to write into) and ``kappa`` (True,
    False or an output tensor [R,C]).  Inputs must stay where they are:
    refill them in place between runs.  Outputs: ``phasors[k]``, ``flags[k]``
    [oR*oC], ``kappa[k]`` (or None)."""

    def __init__(self, items, window, alpha=1e-3, precision="fp32", method="emi", autotune=False):
        lib = load()
        self._keep, self.phasors, self.flags, self.kappa = [], [], [], []
        arr = (_BatchItem * len(items))()
        dev = None
        for k, it in enumerate(items):
            planes = it.get("planes")
            if planes is not None:
                for t in planes:
                    _need(t, torch.complex64, 2, "Batch plane")
                N = len(planes)
                R, C = planes[0].shape
                dev = planes[0].device
                z = None
                parr = (ctypes.c_void_p * N)(*[t.data_ptr() for t in planes])
                self._keep += list(planes) + [parr]
            else:
                z = it["stack"]
                _need(z, torch.complex64, 3, "Batch stack")
                N, R, C = z.shape
                dev = z.device
                parr = None
            oR, oC = output_grid(R, C, window)
            ph = it.get("phasors")
            if ph is None:
                ph = torch.empty((N, oR, oC), dtype=torch.complex64, device=dev)
            elif ph.dtype != torch.complex64 or ph.numel() != N * oR * oC or not ph.is_contiguous():
                raise PlinkError("Batch: phasors must be contiguous complex64 [N,oR,oC]")
            fl = torch.empty((oR * oC,), dtype=torch.uint8, device=dev)
            kap = it.get("kappa", True)
            if kap is True:
                kap = torch.empty((R, C), dtype=torch.complex64, device=dev)
            elif kap is False:
                kap = None
            else:
                _need(kap, torch.complex64, 2, "Batch kappa")
            mean, var = it.get("mean"), it.get("var")
            for t, nm in ((mean, "mean"), (var, "var")):
                if t is not None:
                    _need(t, torch.float64, 2, f"Batch {nm}")
            self._keep += [z, mean, var]
            self.phasors.append(ph)
            self.flags.append(fl)
            self.kappa.append(kap)
            arr[k] = _BatchItem(z.data_ptr() if z is not None else None, R, C, N, int(it.get("first_real", 0)),
                                int(it.get("ref", 0)),
                                mean.data_ptr() if mean is not None else None,
                                var.data_ptr() if var is not None else None, float(it.get("n_eff", 0.0)),
                                ph.data_ptr(), fl.data_ptr(), kap.data_ptr() if kap is not None else None,
                                ctypes.cast(parr, ctypes.POINTER(ctypes.c_void_p)) if parr is not None else None,
                                int(it.get("level", 0)))
        self._device = dev
        h = _P()
        _check(lib.pl_batch_plan(arr, len(items), _win(window), float(alpha), _PREC[precision],
                                 _METHOD[method], 1 if autotune else 0,
                                 _P(torch.cuda.current_stream(dev).cuda_stream), ctypes.byref(h)),
               "Batch plan")
        self._h = h

    def run(self):
        _check(load().pl_batch_run(self._h, _P(torch.cuda.current_stream(self._device).cuda_stream)), "Batch run")

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(8192)
        _check(load().pl_batch_describe(self._h, buf, len(buf)), "Batch describe")
        return buf.value.decode()

    def set_single_launch(self, on: bool):
        """True: each run is one persistent launch over every item and stage
        (the default when the plan supports it); False: one launch per stage
        and kernel variant."""
        _check(load().pl_batch_set_single_launch(self._h, int(bool(on))), "Batch.set_single_launch")

    def set_wait_limit(self, spins: int):
        """Bound of each wait of the single launch (sleep rounds); 0 makes
        every wait give up at once (for tests of the failure path)."""
        _check(load().pl_batch_set_wait_limit(self._h, int(spins)), "Batch.set_wait_limit")

    def check(self):
        """Synchronises and raises if a single-launch run waited past its bound."""
        _check(load().pl_batch_check(self._h, _P(torch.cuda.current_stream(self._device).cuda_stream)),
               "Batch.check")

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().pl_batch_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class SequentialParams:
    R: int
    C: int
    M: int
    K_max: int
    window: tuple
    alpha: float = 1e-3
    precision: str = "fp32"
    method: str = "emi"
    reference: str = "compressed"
    weight_decay: float = 1.0


_REFERENCE = {"compressed": 0, "last": 1}


class Sequential:
    """Sequential estimator (mini-stack reference scheme, compressed SLCs).
    reference="last" forms the compressed SLCs referenced to the last real
    SLC of each mini-stack; weight_decay < 1 weights older statistics
    exponentially less."""

    def __init__(self, R, C, M, K_max, window, alpha=1e-3, precision="fp32", method="emi",
                 device="cuda", reference="compressed", weight_decay=1.0, workspace=None):
        """workspace: optional uint8 device tensor of at least workspace_size(...)
        bytes that holds the driver's device state (the driver then allocates
        nothing; the tensor must outlive it).  Without it the library
        allocates the state itself."""
        lib = load()
        self.params = SequentialParams(R, C, M, K_max, tuple(window), alpha, precision, method, reference,
                                       weight_decay)
        self.device = torch.device(device)
        self.out_shape = output_grid(R, C, window)
        p = _SeqParams(int(R), int(C), int(M), int(K_max), _win(window), float(alpha),
                       _PREC[precision], _METHOD[method], _REFERENCE[reference], float(weight_decay))
        h = _P()
        with torch.cuda.device(self.device):
            if workspace is None:
                _check(lib.pl_seq_create(ctypes.byref(p), ctypes.byref(h)), "Sequential")
            else:
                _need(workspace, torch.uint8, 1, "Sequential(workspace)")
                _check(lib.pl_seq_create_in(ctypes.byref(p), _ptr(workspace), workspace.numel(), ctypes.byref(h)),
                       "Sequential")
        self._ws = workspace
        self._h = h

    @staticmethod
    def workspace_size(R, C, M, K_max, window, alpha=1e-3, precision="fp32", method="emi",
                       reference="compressed", weight_decay=1.0) -> int:
        """Bytes of device state of a driver with these parameters."""
        p = _SeqParams(int(R), int(C), int(M), int(K_max), _win(window), float(alpha),
                       _PREC[precision], _METHOD[method], _REFERENCE[reference], float(weight_decay))
        n = ctypes.c_size_t()
        _check(load().pl_seq_workspace_size(ctypes.byref(p), ctypes.byref(n)), "Sequential.workspace_size")
        return n.value

    def close(self):
        if getattr(self, "_h", None):
            load().pl_seq_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def count(self) -> int:
        c = _I64()
        _check(load().pl_seq_count(self._h, ctypes.byref(c)), "Sequential.count")
        return c.value

    def push(self, new_slcs: torch.Tensor, counters=None, want_kappa=True, want_flags=False):
        """Links the next mini-stack [M,R,C]; returns (phasors [M,oR,oC], kappa [R,C] or None,
        flags [oR,oC] or None)."""
        p = self.params
        _need(new_slcs, torch.complex64, 3, "Sequential.push")
        if tuple(new_slcs.shape) != (p.M, p.R, p.C):
            raise PlinkError("Sequential.push: expected [M,R,C] new SLCs")
        oR, oC = self.out_shape
        ph = torch.empty((p.M, oR, oC), dtype=torch.complex64, device=new_slcs.device)
        kap = torch.empty((p.R, p.C), dtype=torch.complex64, device=new_slcs.device) if want_kappa else None
        fl = torch.empty((oR, oC), dtype=torch.uint8, device=new_slcs.device) if want_flags else None
        _check(load().pl_seq_push(self._h, _ptr(new_slcs), _ptr(ph), _ptr(kap), _ptr(fl),
                                  _ptr(counters), _stream(new_slcs)), "Sequential.push")
        return ph, kap, fl

    def last_mask(self) -> torch.Tensor:
        """SHP masks [oR, oC, nwords] (int32 holding uint32 bits) of the most
        recent mini-stack."""
        oR, oC = self.out_shape
        m = torch.empty((oR, oC, mask_words(self.params.window)), dtype=torch.int32, device=self.device)
        _check(load().pl_seq_last_mask(self._h, _ptr(m), _stream(m)), "Sequential.last_mask")
        return m

    def save(self) -> bytes:
        n = ctypes.c_size_t()
        _check(load().pl_seq_state_size(self._h, ctypes.byref(n)), "Sequential.save")
        buf = ctypes.create_string_buffer(n.value)
        s = _P(torch.cuda.current_stream(self.device).cuda_stream)
        _check(load().pl_seq_save(self._h, buf, n.value, s), "Sequential.save")
        return buf.raw

    def load_state(self, state: bytes):
        buf = ctypes.create_string_buffer(state, len(state))
        s = _P(torch.cuda.current_stream(self.device).cuda_stream)
        _check(load().pl_seq_load(self._h, buf, len(state), s), "Sequential.load_state")
