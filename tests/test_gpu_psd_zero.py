"""PSD values that are not positive and finite at DC and Nyquist (rows the statistic never uses): the transform
writes pixel 0 and weight 0 there, so the statistic kernels, which read the DC row with weight 0 for tracks
whose 21-bin window starts at bin 0, stay finite and equal the oracle's, which skips those rows."""
import numpy as np
import pytest
import torch

import tfsc_inputs as ti
from oracle import cpu as ocpu
from oracle import o2
from oracle import track as otrk
from oracle import transform as otf

from gpu_common import dev, gridspec, lib, note, rel

pytestmark = pytest.mark.gpu


def _data():
    g = ti.custom_grid(2, 512, 300, dt=5.0, modulated=True, gapped=True, cfg_id=9)
    x = ti.noise(g)
    keep, mu = ti.tranche_keep(g), ti.tranche_psd_scale(g)
    dT = g.tranche_dur
    # k_c = ceil(f dT) = 10 puts bin k_c - 10 = 0 in the window; tracks from bin 8.3 to 12 cross it
    b = ti.random_bank(48, 9, mc_range=(5.0, 40.0), f0_range=(8.3 / dT, 12.0 / dT), stream=91)
    b.f0[0] = 9.5 / dT
    return g, x, keep, mu, b


@pytest.mark.parametrize("bad", [0.0, np.inf])
def test_separable_psd_zero_or_inf_at_dc_and_nyquist(bad):
    tfsc = lib()
    g, x, keep, mu, b = _data()
    psd = ti.psd_on_bins(g).copy()
    psd[0] = bad
    psd[-1] = bad
    note(f"psd0 = {bad} at DC and Nyquist; {len(b)} templates near bin 10")
    with np.errstate(divide="ignore", invalid="ignore"):
        pix, u, wm = otf.transform(x, g, psd, mu, keep, 0.1, "rfft")
    ref = ocpu.statistic(pix, u, wm, b, g)
    lay = otrk.Layout(b, g)
    assert np.all(np.isfinite(ref.stat)) and np.max(ref.stat) > 0
    bt = tfsc.BankTensors.from_host(b)
    seg = tfsc.segment_layout(gridspec(g), bt)
    for dtype, layout, precision, schedule, tol in (("f64", "layer", "f64", "wave", 1e-6),
                                                     ("f64", "tranche", "f64", "thread", 1e-6),
                                                     ("f32", "layer_ci", "f32", "wave", 1e-4),
                                                     ("f32", "tranche", "f32", "thread", 1e-4)):
        xs = x if dtype == "f64" else x.astype(np.float32)
        st = tfsc.transform(gridspec(g), dev(xs), dev(psd), dev(mu), dev(keep), dtype=dtype, layout=layout)
        assert torch.isfinite(st.pix).all(), (dtype, layout)
        assert float(st.inv_asd[0]) == 0.0 and float(st.inv_asd[-1]) == 0.0
        res = tfsc.bank_statistic(gridspec(g), st, bt, seg, precision=precision, schedule=schedule)
        s = res.stat.cpu().numpy()
        r = rel(s, ref.stat)
        note(f"  {schedule} {dtype} {layout}: max rel {r.max():.2e}")
        assert np.all(np.isfinite(s)), (schedule, dtype)
        assert r.max() < tol, (schedule, dtype, r.max())
        assert np.array_equal(res.flags.cpu().numpy(), ref.flags)
    assert np.array_equal(lay.nseg, seg.nseg.cpu().numpy())


def test_per_pixel_psd_zero_at_dc_and_nyquist():
    tfsc = lib()
    g, x, keep, mu, b = _data()
    S = ti.tranche_psd_tf(g).copy()
    S[0, :] = 0.0
    S[-1, :] = 0.0
    note("per-pixel PSD 0 at DC and Nyquist")
    with np.errstate(divide="ignore", invalid="ignore"):
        pix, wt = otf.transform_tf(x, g, S, keep, 0.1, "rfft")
        ref = o2.statistic(pix, None, None, b, g, layout=otrk.Layout(b, g), weight_tf=wt)
    bt = tfsc.BankTensors.from_host(b)
    seg = tfsc.segment_layout(gridspec(g), bt)
    for dtype, layout, schedule, tol in (("f64", "layer", "wave", 1e-6), ("f32", "layer_ci", "wave", 1e-4),
                                         ("f32", "tranche", "thread", 1e-4)):
        xs = x if dtype == "f64" else x.astype(np.float32)
        st = tfsc.transform_tf(gridspec(g), dev(xs), dev(S), dev(keep), dtype=dtype, layout=layout)
        assert torch.isfinite(st.pix).all() and torch.isfinite(st.rho).all()
        assert float(st.inv_asd[0]) == 0.0
        res = tfsc.bank_statistic(gridspec(g), st, bt, seg, precision=dtype, schedule=schedule)
        s = res.stat.cpu().numpy()
        r = rel(s, ref.stat)
        note(f"  {schedule} {dtype} {layout}: max rel {r.max():.2e}")
        assert np.all(np.isfinite(s))
        assert r.max() < tol, (schedule, dtype, r.max())
        assert np.array_equal(res.flags.cpu().numpy(), ref.flags)
