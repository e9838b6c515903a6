"""The C ABI library: it loads, exports every symbol the header declares, and
its host-side checks reject bad arguments before touching a GPU (no compute
call is made here)."""
import ctypes
import os
import re

import pytest

import paper_2511_12051_amd as plink

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "plink.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pl_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(plink.library_path()):
        pytest.fail("libplink.so is not built (python -m paper_2511_12051_amd.build)")
    return plink.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    # and the binding declares a signature for each of them
    assert set(names) == set(plink._SIGNATURES)


def test_status_strings_and_version(lib):
    assert lib.pl_version().decode().startswith("plink")
    for s in range(7):
        assert lib.pl_status_string(s).decode()
    assert lib.pl_status_string(99).decode() == "unknown status"


def test_output_grid_and_mask_words():
    assert plink.output_grid(2048, 8192, (11, 5, 6, 3)) == (682, 1365)
    assert plink.output_grid(64, 64, (5, 5, 1, 1)) == (64, 64)
    assert plink.output_grid(10, 14, (2, 1, 4, 3)) == (3, 3)
    assert plink.mask_words((11, 5, 6, 3)) == 8
    assert plink.mask_words((19, 9, 6, 3)) == 24
    with pytest.raises(plink.PlinkError):
        plink.mask_words((16, 16, 1, 1))  # 33 x 33 = 1089 > PL_MAX_WINDOW
    with pytest.raises(plink.PlinkError):
        plink.output_grid(0, 5, (1, 1, 1, 1))


def _w(*v):
    return plink._Window(*v)


def test_argument_errors_return_before_any_device_work(lib):
    P = ctypes.c_void_p
    fake = P(0x1000)  # never dereferenced: every call below fails its checks first
    # NULL pointers
    assert lib.pl_amplitude_stats(None, 5, 4, 4, fake, fake, None) == 1
    assert lib.pl_shp_select(fake, fake, 8, 8, 10.0, _w(1, 1, 1, 1), 1e-3, None, fake, None, None) == 1
    # N outside 1..32
    assert lib.pl_estimate_coherence(fake, 33, 8, 8, _w(1, 1, 1, 1), fake, 0, fake, None) == 3
    assert lib.pl_phase_link(fake, 0, 10, 0, 0, fake, None, None, None, None, None, None) == 3
    assert lib.pl_phase_link(None, 5, 0, 0, 0, None, None, None, None, None, None, None) == 0
    assert lib.pl_amplitude_stats(fake, 40, 4, 4, fake, fake, None) == 3
    # bad window / shapes
    assert lib.pl_shp_select(fake, fake, 8, 8, 10.0, _w(-1, 1, 1, 1), 1e-3, fake, fake, None, None) == 2
    assert lib.pl_shp_select(fake, fake, 2, 2, 10.0, _w(1, 1, 3, 3), 1e-3, fake, fake, None, None) == 2
    # bad scalars
    assert lib.pl_shp_select(fake, fake, 8, 8, 0.0, _w(1, 1, 1, 1), 1e-3, fake, fake, None, None) == 1
    assert lib.pl_shp_select(fake, fake, 8, 8, 5.0, _w(1, 1, 1, 1), 1.5, fake, fake, None, None) == 1
    assert lib.pl_phase_link(fake, 5, 10, 5, 0, fake, None, None, None, None, None, None) == 1
    assert lib.pl_phase_link(fake, 5, 10, 0, 7, fake, None, None, None, None, None, None) == 1
    assert lib.pl_estimate_coherence(fake, 5, 8, 8, _w(1, 1, 1, 1), fake, 9, fake, None) == 1
    assert lib.pl_compress_ministack(fake, 5, 5, 8, 8, _w(1, 1, 1, 1), fake, fake, None) == 1
    # adjoint: workspace size, too-small workspace, bad reference
    n = ctypes.c_size_t()
    assert lib.pl_phase_link_vjp_workspace(20, 64, 64, _w(7, 7, 1, 1), ctypes.byref(n)) == 0
    P, N = 64 * 64, 20
    assert n.value >= P * N * N * 8 + P * N * 4 + P * (N * (N + 1) // 2) * 8
    assert lib.pl_phase_link_vjp(fake, 20, 64, 64, _w(7, 7, 1, 1), fake, fake, 0, 0, fake, fake, fake,
                                 n.value - 1, None) == 5
    assert lib.pl_phase_link_vjp(fake, 20, 64, 64, _w(7, 7, 1, 1), fake, fake, 20, 0, fake, fake, fake,
                                 n.value, None) == 1
    assert lib.pl_phase_link_vjp(fake, 40, 64, 64, _w(7, 7, 1, 1), fake, fake, 0, 0, fake, fake, fake,
                                 n.value, None) == 3
    assert lib.pl_phase_link_vjp(None, 20, 64, 64, _w(7, 7, 1, 1), fake, fake, 0, 0, fake, fake, fake,
                                 n.value, None) == 1
    w = (ctypes.c_double * 2)(1.0, -1.0)
    assert lib.pl_merge_amplitude_stats(fake, fake, w, 2, 4, 4, fake, fake, None) == 1
    # fused coherence + linking: one output row of packed matrices at least
    lo, hi = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.pl_phase_link_fused_workspace(25, 96, 384, _w(11, 5, 6, 3), ctypes.byref(lo), ctypes.byref(hi)) == 0
    assert lo.value == 64 * 325 * 8 and hi.value == 32 * lo.value
    args = [fake, 25, 96, 384, _w(11, 5, 6, 3), fake, 1, 9, 0, fake, None, None, None, None, None, fake]
    assert lib.pl_phase_link_fused(*args, lo.value - 1, None) == 5
    assert lib.pl_phase_link_fused(*args[:15], None, lo.value, None) == 1
    bad = list(args)
    bad[7] = 25  # reference outside 0..N-1
    assert lib.pl_phase_link_fused(*bad, lo.value, None) == 1
    bad = list(args)
    bad[1] = 33
    assert lib.pl_phase_link_fused(*bad, lo.value, None) == 3
    assert lib.pl_sync_report(None, None, None) == 1
    # empty pixel list is a no-op
    assert lib.pl_phase_link(fake, 5, 0, 0, 0, fake, None, None, None, None, None, None) == 0
    assert "ref_idx" in lib.pl_last_error().decode() or lib.pl_last_error() is not None


def test_sequential_parameter_checks(lib):
    p = plink._SeqParams(64, 64, 20, 13, _w(2, 2, 1, 1), 1e-3, 0, 0)  # M + K_max > 32
    h = ctypes.c_void_p()
    assert lib.pl_seq_create(ctypes.byref(p), ctypes.byref(h)) == 3
    p = plink._SeqParams(64, 64, 15, 6, _w(2, 2, 1, 1), 2.0, 0, 0)
    assert lib.pl_seq_create(ctypes.byref(p), ctypes.byref(h)) == 1
    p = plink._SeqParams(64, 64, 15, 6, _w(2, 2, 1, 1), 1e-3, 0, 0, 2)  # unknown reference mode
    assert lib.pl_seq_create(ctypes.byref(p), ctypes.byref(h)) == 1
    for decay in (0.0, 1.5, float("nan")):
        p = plink._SeqParams(64, 64, 15, 6, _w(2, 2, 1, 1), 1e-3, 0, 0, 1, decay)
        assert lib.pl_seq_create(ctypes.byref(p), ctypes.byref(h)) == 1
    assert lib.pl_seq_destroy(None) == 0


def test_product_argument_checks(lib):
    P = ctypes.c_void_p
    fake = P(0x1000)
    n = ctypes.c_int32()
    assert lib.pl_network_size(15, 3, ctypes.byref(n)) == 0 and n.value == 39
    assert lib.pl_network_size(32, 3, ctypes.byref(n)) == 0 and n.value == 90
    assert lib.pl_network_size(15, 4, ctypes.byref(n)) == 3
    assert lib.pl_network_size(1, 3, ctypes.byref(n)) == 3
    assert lib.pl_network_invert_l1(fake, 15, 3, 100, 0.0, 10, fake, None, None) == 1  # rho
    assert lib.pl_network_invert_l1(fake, 15, 3, 100, 1.0, -1, fake, None, None) == 1  # iterations
    assert lib.pl_network_invert_l1(None, 15, 3, 0, 1.0, 10, None, None, None) == 0   # no pixels
    assert lib.pl_phase_similarity(fake, 15, 10, 10, None, 16, 3, fake, None) == 3      # radius
    assert lib.pl_phase_similarity(fake, 15, 10, 10, None, 3, 4, fake, None) == 3       # network
    assert lib.pl_phase_similarity(None, 15, 10, 10, None, 3, 3, fake, None) == 1
    w = _w(11, 5, 6, 3)
    assert lib.pl_ps_regrid(fake, 15, 96, 384, w, 15, fake, fake, 0.2, fake, fake, None, None, None) == 1
    assert lib.pl_ps_regrid(fake, 15, 96, 384, w, 0, fake, fake, -0.2, fake, fake, None, None, None) == 1
    assert lib.pl_ps_regrid(fake, 15, 96, 384, w, 0, None, fake, 0.2, fake, fake, None, None, None) == 1


def test_binding_refuses_cpu_tensors():
    import torch
    x = torch.zeros((3, 4, 4), dtype=torch.complex64)
    with pytest.raises(plink.PlinkError):
        plink.amplitude_stats(x)


def test_batch_argument_checks(lib):
    P = ctypes.c_void_p
    fake = 0x1000  # never dereferenced: every call below fails its checks first
    h = P()
    item = plink._BatchItem(fake, 64, 64, 15, 0, 0, None, None, 0.0, fake, None, None, None, 0)
    items = (plink._BatchItem * 1)(item)
    w = _w(5, 5, 1, 1)
    assert lib.pl_batch_plan(None, 1, w, 1e-3, 0, 0, 0, None, ctypes.byref(h)) == 1
    assert lib.pl_batch_plan(items, 0, w, 1e-3, 0, 0, 0, None, ctypes.byref(h)) == 3
    assert lib.pl_batch_plan(items, 1, w, 1.5, 0, 0, 0, None, ctypes.byref(h)) == 1
    for bad in (dict(N=40), dict(first_real=15), dict(ref_idx=-1), dict(stack=None), dict(R=0)):
        it = plink._BatchItem(fake, 64, 64, 15, 0, 0, None, None, 0.0, fake, None, None, None, 0)
        for k, v in bad.items():
            setattr(it, k, v)
        arr = (plink._BatchItem * 1)(it)
        assert lib.pl_batch_plan(arr, 1, w, 1e-3, 0, 0, 0, None, ctypes.byref(h)) != 0, bad
    it = plink._BatchItem(fake, 64, 64, 15, 0, 0, fake, None, 0.0, fake, None, None, None, 0)  # mean without var
    assert lib.pl_batch_plan((plink._BatchItem * 1)(it), 1, w, 1e-3, 0, 0, 0, None, ctypes.byref(h)) == 1
    # a plane list with a NULL plane
    planes = (ctypes.c_void_p * 15)(*([fake] * 14 + [None]))
    it = plink._BatchItem(None, 64, 64, 15, 0, 0, None, None, 0.0, fake, None, None,
                          ctypes.cast(planes, ctypes.POINTER(ctypes.c_void_p)), 0)
    assert lib.pl_batch_plan((plink._BatchItem * 1)(it), 1, w, 1e-3, 0, 0, 0, None, ctypes.byref(h)) == 1
    assert lib.pl_batch_destroy(None) == 0
    assert lib.pl_batch_run(None, None) == 1


def test_sequential_workspace_size_and_checks(lib):
    """The driver's device state in one block: its size is a host query, it
    grows with K_max exactly by the compressed-SLC ring and one more set of
    statistics, and creating a driver in a too-small or misaligned buffer is
    rejected before any device work."""
    w = (11, 5, 6, 3)
    R, C, M = 96, 198, 15
    n0 = plink.Sequential.workspace_size(R, C, M, 0, w)
    n2 = plink.Sequential.workspace_size(R, C, M, 2, w)
    oR, oC = plink.output_grid(R, C, w)
    px, P = R * C, oR * oC

    def up(v):
        return (v + 255) // 256 * 256

    # K_max = 2 adds the ring of two compressed SLCs, two more statistics
    # planes pairs, and the wider coherence and phasors of N = M + 2
    grow = up(2 * px * 8) + 2 * up(px * 8 * 3) - 2 * up(px * 8) \
        + up(P * (M + 2) ** 2 * 8) - up(P * M * M * 8) + up(P * (M + 2) * 8) - up(P * M * 8)
    assert n2 - n0 == grow
    p = plink._SeqParams(R, C, M, 2, plink._win(w), 1e-3, 0, 0, 0, 1.0)
    h = plink._P()
    fake = ctypes.c_void_p(0x1000)
    assert lib.pl_seq_create_in(ctypes.byref(p), fake, n2 - 1, ctypes.byref(h)) == 5   # PL_ERR_WORKSPACE
    assert lib.pl_seq_create_in(ctypes.byref(p), ctypes.c_void_p(0x1010), n2, ctypes.byref(h)) == 1  # misaligned
    assert lib.pl_seq_create_in(ctypes.byref(p), None, n2, ctypes.byref(h)) == 1
    bad = plink._SeqParams(R, C, 0, 2, plink._win(w), 1e-3, 0, 0, 0, 1.0)
    n = ctypes.c_size_t()
    assert lib.pl_seq_workspace_size(ctypes.byref(bad), ctypes.byref(n)) == 3
