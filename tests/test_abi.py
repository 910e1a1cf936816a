"""The C-ABI library loads, exports every declared symbol, and validates arguments on the host (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "tfsc.h")) as fh:
        src = fh.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tfsc_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2510_19047_amd import _lib
    return _lib.load()


def test_every_declared_function_is_exported(L):
    names = _declared()
    assert {"tfsc_transform", "tfsc_bank_statistic", "tfsc_statistic_vjp", "tfsc_segment_layout"} <= set(names)
    for n in names:
        assert hasattr(L, n), n
    from paper_2510_19047_amd import _lib
    assert set(_lib.EXPORTS) == set(names)


def test_version_and_status_strings(L):
    assert L.tfsc_abi_version() == 4
    for s in range(8):
        assert len(L.tfsc_status_string(s)) > 0


def _grid(**kw):
    from paper_2510_19047_amd import _lib
    g = dict(n_channels=2, tranche_len=2048, n_tranches=6144, n_fresnel=21, dt=5.0, tukey_alpha=0.1)
    g.update(kw)
    return _lib.Grid(**g)


def test_workspace_sizes(L):
    from paper_2510_19047_amd import _lib
    g = _grid()
    assert L.tfsc_workspace_bytes(ctypes.byref(g), 1_000_000, None, _lib.WS_LAYOUT) >= 8 * (1_000_000 // 256)
    assert L.tfsc_workspace_bytes(ctypes.byref(g), 10, None, _lib.WS_STATISTIC) >= 18 * 8 * 6144
    assert L.tfsc_workspace_bytes(ctypes.byref(g), 0, None, _lib.WS_TRANSFORM) >= 2 * 1025 * 6144 * 8
    bad = _grid(n_fresnel=20)
    assert L.tfsc_workspace_bytes(ctypes.byref(bad), 10, None, _lib.WS_STATISTIC) == 0


def test_argument_errors_return_codes(L):
    from paper_2510_19047_amd import _lib
    g = _grid()
    bank = _lib.Bank(5)  # NULL arrays
    seg = _lib.Segments(0, None, None)
    assert L.tfsc_segment_layout(None, ctypes.byref(bank), ctypes.byref(seg), None, 0, None) == 1
    assert L.tfsc_segment_layout(ctypes.byref(g), ctypes.byref(bank), ctypes.byref(seg), None, 0, None) == 1
    assert L.tfsc_segment_layout(ctypes.byref(_grid(tranche_len=1000)), ctypes.byref(bank), ctypes.byref(seg),
                                 None, 0, None) == 2
    assert L.tfsc_segment_layout(ctypes.byref(_grid(n_fresnel=11)), ctypes.byref(bank), ctypes.byref(seg),
                                 None, 0, None) == 5
    pix = _lib.Pixels(7, 0, None, None, None, None)
    assert L.tfsc_bank_statistic(ctypes.byref(g), ctypes.byref(pix), ctypes.byref(_lib.Bank(0)), ctypes.byref(seg),
                                 None, None, None, None, None, None, None, 0, None) == 3
    pix = _lib.Pixels(5, 0, None, None, None, None)  # one past the last element type (I16 = 4)
    assert L.tfsc_bank_statistic(ctypes.byref(g), ctypes.byref(pix), ctypes.byref(_lib.Bank(0)), ctypes.byref(seg),
                                 None, None, None, None, None, None, None, 0, None) == 3
    assert L.tfsc_track(ctypes.byref(g), ctypes.byref(bank), None, None) == 1


def test_vjp_argument_errors(L):
    from paper_2510_19047_amd import _lib
    g = _grid()
    bank = _lib.Bank(0)
    seg = _lib.Segments(0, None, None)
    pix = _lib.Pixels(1, 0, None, None, None, None)
    # missing pixel weights
    assert L.tfsc_statistic_vjp(ctypes.byref(g), ctypes.byref(pix), ctypes.byref(bank), ctypes.byref(seg), None,
                                None, None, None, None, None, 0, None) == 1
    # an empty bank needs no workspace beyond the declared size, but a NULL workspace is refused
    one = (ctypes.c_double * 4)()
    pix = _lib.Pixels(1, 0, None, None, ctypes.cast(one, ctypes.c_void_p), ctypes.cast(one, ctypes.c_void_p))
    assert L.tfsc_statistic_vjp(ctypes.byref(g), ctypes.byref(pix), ctypes.byref(bank), ctypes.byref(seg), None,
                                None, None, None, None, None, 0, None) == 4


def test_launch_shape_limits(L):
    """block_waves above 4 (256 threads, the kernels' launch bound) is refused before any launch."""
    from paper_2510_19047_amd import _lib
    g = _grid()
    one = (ctypes.c_double * 4)()
    p = ctypes.cast(one, ctypes.c_void_p)
    pix = _lib.Pixels(1, 0, p, None, p, p)
    seg = _lib.Segments(0, p, p)
    bank = _lib.Bank(1, p, p, p, p, p, p, p)
    for bw, gpc in ((5, 1), (8, 2), (1, 65)):
        opt = _lib.Options(1, 1, bw, gpc, None)
        assert L.tfsc_bank_statistic(ctypes.byref(g), ctypes.byref(pix), ctypes.byref(bank), ctypes.byref(seg),
                                     ctypes.byref(opt), p, p, None, p, None, p, 1 << 30, None) == 1


def test_transform_tf_and_channel_argument_errors(L):
    """Host-side checks of the per-pixel PSD transform and of the channel count (no device call is made)."""
    from paper_2510_19047_amd import _lib
    g = _grid()
    dummy = ctypes.c_double(1.0)
    keep = ctypes.c_uint8(1)
    # a store without rho: invalid argument
    pix = _lib.Pixels(1, 0, ctypes.addressof(dummy), None, ctypes.addressof(dummy), ctypes.addressof(dummy), None)
    assert L.tfsc_transform_tf(ctypes.byref(g), ctypes.addressof(dummy), 1, ctypes.addressof(dummy),
                               ctypes.addressof(keep), ctypes.byref(pix), None, 0, None) == 1
    # FP64 store from FP32 samples: unsupported element-type combination
    pix = _lib.Pixels(0, 0, ctypes.addressof(dummy), None, ctypes.addressof(dummy), ctypes.addressof(dummy),
                      ctypes.addressof(dummy))
    assert L.tfsc_transform_tf(ctypes.byref(g), ctypes.addressof(dummy), 1, ctypes.addressof(dummy),
                               ctypes.addressof(keep), ctypes.byref(pix), None, 0, None) == 3
    # no PSD
    assert L.tfsc_transform_tf(ctypes.byref(g), ctypes.addressof(dummy), 0, None, ctypes.addressof(keep),
                               ctypes.byref(pix), None, 0, None) == 1
    # one to three channels; four is a shape error
    assert L.tfsc_workspace_bytes(ctypes.byref(_grid(n_channels=3)), 10, None, _lib.WS_STATISTIC) > 0
    assert L.tfsc_workspace_bytes(ctypes.byref(_grid(n_channels=4)), 10, None, _lib.WS_STATISTIC) == 0
    bank = _lib.Bank(5)
    seg = _lib.Segments(0, None, None)
    assert L.tfsc_segment_layout(ctypes.byref(_grid(n_channels=4)), ctypes.byref(bank), ctypes.byref(seg), None, 0,
                                 None) == 2


def test_transform_tf_binding_checks_the_psd_shape():
    import torch
    import paper_2510_19047_amd as tfsc
    grid = tfsc.GridSpec(2, 512, 100, 5.0, 0.1)
    x = torch.zeros((2, 512 * 100), dtype=torch.float32)
    keep = torch.ones(100, dtype=torch.uint8)
    with pytest.raises(tfsc.TfscError):
        tfsc.transform_tf(grid, x, torch.ones((100, 257), dtype=torch.float64), keep)  # transposed
    with pytest.raises(tfsc.TfscError):
        tfsc.transform_tf(grid, x, torch.ones((257, 100), dtype=torch.float32), keep)  # not float64


def test_abi3_argument_errors(L):
    """Host-side checks of the version-3 additions: the bank's ln_mc, the Fresnel mode, the multi-harmonic call,
    the orbit positions and the tuner (no device call is made)."""
    from paper_2510_19047_amd import _lib
    g = _grid()
    one = (ctypes.c_double * 4)()
    p = ctypes.cast(one, ctypes.c_void_p)
    pix = _lib.Pixels(1, 0, p, None, p, p, None, None)
    seg = _lib.Segments(0, p, p)
    ws = 1 << 30
    # exactly one of mc and ln_mc
    both = _lib.Bank(1, p, p, p, p, p, p, p, p)
    neither = _lib.Bank(1, None, p, p, p, p, p, p, None)
    for bank in (both, neither):
        assert L.tfsc_bank_statistic(ctypes.byref(g), ctypes.byref(pix), ctypes.byref(bank), ctypes.byref(seg),
                                     None, p, p, None, p, None, p, ws, None) == 1
        assert L.tfsc_segment_layout(ctypes.byref(g), ctypes.byref(bank), ctypes.byref(seg), p, ws, None) == 1
    bank = _lib.Bank(1, None, p, p, p, p, p, p, p)  # ln_mc only: valid
    # Fresnel mode out of range; the accurate mode with F32 pixels and F64 arithmetic, or with 16-bit pixels
    assert L.tfsc_bank_statistic(ctypes.byref(g), ctypes.byref(pix), ctypes.byref(bank), ctypes.byref(seg),
                                 ctypes.byref(_lib.Options(1, 1, 0, 0, None, 2, None)), p, p, None, p, None, p, ws,
                                 None) == 1
    assert L.tfsc_bank_statistic(ctypes.byref(g), ctypes.byref(pix), ctypes.byref(bank), ctypes.byref(seg),
                                 ctypes.byref(_lib.Options(0, 0, 0, 0, None, 1, None)), p, p, None, p, None, p, ws,
                                 None) == 5
    pix16 = _lib.Pixels(3, 0, p, p, p, p, None, None)
    assert L.tfsc_bank_statistic(ctypes.byref(g), ctypes.byref(pix16), ctypes.byref(bank), ctypes.byref(seg),
                                 ctypes.byref(_lib.Options(1, 1, 0, 0, None, 1, None)), p, p, None, p, None, p, ws,
                                 None) == 5
    # the int16 fixed-point store: needs its layer scales, takes FP32 arithmetic only
    pixi = _lib.Pixels(4, 0, p, None, p, p, None, None)
    assert L.tfsc_bank_statistic(ctypes.byref(g), ctypes.byref(pixi), ctypes.byref(bank), ctypes.byref(seg),
                                 ctypes.byref(_lib.Options(1, 1, 0, 0, None, 0, None)), p, p, None, p, None, p, ws,
                                 None) == 1
    pixi = _lib.Pixels(4, 0, p, p, p, p, None, None)
    assert L.tfsc_bank_statistic(ctypes.byref(g), ctypes.byref(pixi), ctypes.byref(bank), ctypes.byref(seg),
                                 ctypes.byref(_lib.Options(0, 1, 0, 0, None, 0, None)), p, p, None, p, None, p, ws,
                                 None) == 3
    # the VJP takes the paper's Fresnel forms only
    assert L.tfsc_statistic_vjp(ctypes.byref(g), ctypes.byref(pix), ctypes.byref(bank), ctypes.byref(seg),
                                ctypes.byref(_lib.Options(1, 1, 0, 0, None, 1, None)), p, p, None, p, p, ws,
                                None) == 5
    # harmonics: count, range, duplicates, schedule, per-pixel PSD
    opt = _lib.Options(1, 1, 0, 0, None, 0, None)

    def harm(hs, o=opt, px=pix):
        arr = (ctypes.c_int32 * max(len(hs), 1))(*hs)
        return L.tfsc_bank_statistic_harmonics(ctypes.byref(g), ctypes.byref(px), ctypes.byref(bank),
                                               ctypes.byref(seg), ctypes.byref(o), len(hs), arr, p, p, p, None, p,
                                               None, p, ws, None)

    assert harm([]) == 1
    assert harm([1, 2, 3, 4, 5]) == 1
    assert harm([2, 2]) == 1
    assert harm([9]) == 1 and harm([0, 2]) == 1
    assert harm([1, 2], o=_lib.Options(1, 0, 0, 0, None, 0, None)) == 5
    assert harm([1, 2], px=_lib.Pixels(1, 0, p, None, p, p, p, None)) == 5
    assert harm([1, 2], o=_lib.Options(0, 1, 0, 0, None, 0, None)) == 3
    # orbit positions and tuner arguments
    assert L.tfsc_orbit_positions(ctypes.byref(g), None, None) == 1
    bw, gpc = ctypes.c_int32(), ctypes.c_int32()
    assert L.tfsc_tune_statistic(ctypes.byref(g), ctypes.byref(pix), ctypes.byref(bank), ctypes.byref(seg), None,
                                 None, p, p, p, p, ws, None, ctypes.byref(bw), ctypes.byref(gpc)) == 1


def test_links_argument_errors(L):
    """Host-side checks of the link light-time table (tfsc_pixels.links): the statistic takes it with F64 or F32
    pixels in the same arithmetic, no rho and the paper's Fresnel forms; the VJP, the several-realisation and the
    harmonics calls refuse it; tfsc_link_lengths needs its output (no device call is made)."""
    from paper_2510_19047_amd import _lib
    g = _grid()
    one = (ctypes.c_double * 4)()
    p = ctypes.cast(one, ctypes.c_void_p)
    seg = _lib.Segments(0, p, p)
    bank = _lib.Bank(1, p, p, p, p, p, p, p, None)
    ws = 1 << 30

    def stat(px, o):
        return L.tfsc_bank_statistic(ctypes.byref(g), ctypes.byref(px), ctypes.byref(bank), ctypes.byref(seg),
                                     ctypes.byref(o), p, p, None, p, None, p, ws, None)

    f32 = _lib.Options(1, 1, 0, 0, None, 0, None)
    lk = _lib.Pixels(1, 2, p, None, p, p, None, None, p)
    assert stat(_lib.Pixels(1, 2, p, None, p, p, p, None, p), f32) == 5  # with rho
    assert stat(lk, _lib.Options(1, 1, 0, 0, None, 1, None)) == 5  # accurate Fresnel mode
    assert stat(lk, _lib.Options(0, 1, 0, 0, None, 0, None)) == 5  # F32 pixels, F64 arithmetic
    assert stat(_lib.Pixels(4, 2, p, p, p, p, None, None, p), f32) == 5  # int16 store
    assert L.tfsc_statistic_vjp(ctypes.byref(g), ctypes.byref(lk), ctypes.byref(bank), ctypes.byref(seg),
                                ctypes.byref(f32), p, p, None, p, p, ws, None) == 5
    assert L.tfsc_bank_statistic_multi(ctypes.byref(g), ctypes.byref(lk), 2, 0, 0, ctypes.byref(bank),
                                       ctypes.byref(seg), ctypes.byref(f32), 0, p, p, p, None, p, ws, None) == 5
    arr = (ctypes.c_int32 * 1)(2)
    assert L.tfsc_bank_statistic_harmonics(ctypes.byref(g), ctypes.byref(lk), ctypes.byref(bank), ctypes.byref(seg),
                                           ctypes.byref(f32), 1, arr, p, p, p, None, p, None, p, ws, None) == 5
    assert L.tfsc_link_lengths(ctypes.byref(g), None, None, None) == 1
    assert L.tfsc_link_lengths(ctypes.byref(_grid(n_tranches=0)), None, p, None) != 0


def test_tdi_generation_argument_errors(L):
    """tfsc_pixels.tdi_generation: 0, 1 or 2, and 2 only with the link light-time table (no device call)."""
    from paper_2510_19047_amd import _lib
    g = _grid()
    one = (ctypes.c_double * 4)()
    p = ctypes.cast(one, ctypes.c_void_p)
    seg = _lib.Segments(0, p, p)
    bank = _lib.Bank(1, p, p, p, p, p, p, p, None)
    opt = _lib.Options(1, 1, 0, 0, None, 0, None)

    def stat(px):
        return L.tfsc_bank_statistic(ctypes.byref(g), ctypes.byref(px), ctypes.byref(bank), ctypes.byref(seg),
                                     ctypes.byref(opt), p, p, None, p, None, p, 1 << 30, None)

    assert stat(_lib.Pixels(1, 2, p, None, p, p, None, None, p, 3)) == 1
    assert stat(_lib.Pixels(1, 2, p, None, p, p, None, None, p, -1)) == 1
    assert stat(_lib.Pixels(1, 2, p, None, p, p, None, None, None, 2)) == 5
