"""Multi-harmonic templates (Sec. "Outlook": {A, f, fdot, phi} for each harmonic and the Fresnel expressions
applied to each) through the C ABI, against the oracle (``oracle.harmonics``).

Data: two channels with gaps and modulation, noise plus a pixel-domain injection of a three-harmonic signal.
The bank mixes templates whose harmonic windows overlap (below ~16 mHz on this grid, where the orbital
frequency is under 21 bins) with ones whose windows are disjoint, an invalid row and the exact injection.
"""
import functools

import numpy as np
import pytest
import torch

import tfsc_inputs as ti
from oracle import harmonics as oh
from oracle import transform as otf

from gpu_common import dev, gridspec, lib, note, rel

pytestmark = pytest.mark.gpu

HS = [1, 2, 3]


@functools.lru_cache(maxsize=2)
def _data(n_channels=2):
    g = ti.custom_grid(n_channels, 512, 300, dt=5.0, modulated=True, gapped=True, cfg_id=21)
    psd, mu, keep = ti.psd_on_bins(g), ti.tranche_psd_scale(g), ti.tranche_keep(g)
    pix, u, wm = otf.transform(ti.noise(g), g, psd, mu, keep, 0.1, "rfft")
    b = ti.random_bank(40, 21, mc_range=(5.0, 60.0), f0_range=(0.004, 0.06), eta=None, stream=41)
    b.mc[5] = -1.0  # invalid
    rng = np.random.default_rng(21)
    amps = (rng.normal(size=(40, 3)) + 1j * rng.normal(size=(40, 3))) * np.array([0.3, 1.0, 0.4])
    amps[:, 1] = 1.0
    # inject template 0 (f0 in the overlapping range) with its own harmonics, SNR 25
    b.f0[0] = 0.009
    Y = oh.template_column_pixels(b, 0, g, u, wm, HS, amps[0])
    rho = np.sqrt(2.0 * np.sum(np.abs(Y[:, 1:-1]) ** 2))
    pix = pix + Y * (25.0 / rho)
    return g, pix, u, wm, b, amps


def _amp_dev(amps):
    return dev(np.ascontiguousarray(amps.astype(np.complex128)))


@pytest.mark.parametrize("dtype,layout,tol", [("f64", "layer", 1e-6), ("f64", "layer_ci", 1e-6),
                                              ("f32", "layer_ci", 1e-4)])
def test_harmonics_against_the_oracle(dtype, layout, tol):
    tfsc = lib()
    g, pix, u, wm, b, amps = _data()
    note(f"harmonics {HS}: {dtype} {layout}")
    ref = oh.statistic(pix, u, wm, b, g, HS, amps)
    bt = tfsc.BankTensors.from_host(b)
    seg = tfsc.segment_layout(gridspec(g), bt)
    store = tfsc.PixelStore.from_complex(dev(pix), dev(u), dev(wm), dtype=dtype, layout=layout)
    res = tfsc.bank_statistic_harmonics(gridspec(g), store, bt, seg, HS, _amp_dev(amps), precision=dtype,
                                        want_active=True)
    s = res.stat.cpu().numpy()
    r = rel(s, ref.stat)
    st = res.seg_terms.cpu().numpy()[: seg.total]
    rs = np.abs(st - ref.seg_terms) / np.maximum(ref.seg_terms, 1.0)
    note(f"  max rel {r.max():.2e} (segment terms {rs.max():.2e}); injection {s[0]:.2f} vs oracle {ref.stat[0]:.2f}")
    assert np.array_equal(res.flags.cpu().numpy(), ref.flags)
    assert r.max() < tol and rs.max() < tol
    assert int(np.argmax(s)) == 0


def test_dominant_harmonic_alone_is_the_statistic():
    tfsc = lib()
    g, pix, u, wm, b, amps = _data()
    bt = tfsc.BankTensors.from_host(b)
    seg = tfsc.segment_layout(gridspec(g), bt)
    store = tfsc.PixelStore.from_complex(dev(pix), dev(u), dev(wm), dtype="f64", layout="layer_ci")
    a = tfsc.bank_statistic(gridspec(g), store, bt, seg, precision="f64", schedule="wave")
    h = tfsc.bank_statistic_harmonics(gridspec(g), store, bt, seg, [2], torch.ones((bt.n, 1), dtype=torch.complex128,
                                                                                  device="cuda"), precision="f64")
    r = rel(h.stat.cpu().numpy(), a.stat.cpu().numpy())
    note(f"harmonic 2 alone vs the single-harmonic kernel: max rel {r.max():.2e}")
    assert r.max() < 1e-12
    assert torch.equal(h.flags, a.flags)


def test_three_channels_with_harmonics():
    tfsc = lib()
    g, pix, u, wm, b, amps = _data(3)
    ref = oh.statistic(pix, u, wm, b, g, HS, amps)
    bt = tfsc.BankTensors.from_host(b)
    seg = tfsc.segment_layout(gridspec(g), bt)
    store = tfsc.PixelStore.from_complex(dev(pix), dev(u), dev(wm), dtype="f64", layout="layer_ci")
    res = tfsc.bank_statistic_harmonics(gridspec(g), store, bt, seg, HS, _amp_dev(amps), precision="f64")
    r = rel(res.stat.cpu().numpy(), ref.stat)
    note(f"harmonics, A + E + T: max rel {r.max():.2e}")
    assert r.max() < 1e-6
    assert np.array_equal(res.flags.cpu().numpy(), ref.flags)


def test_harmonics_of_a_bank_given_in_ln_mc():
    tfsc = lib()
    g, pix, u, wm, b, amps = _data()
    bt = tfsc.BankTensors.from_host(b)
    # ln of the invalid row's negative mass is NaN: that row stays invalid
    bl = tfsc.BankTensors(None, bt.eta, bt.f0, bt.cos_theta, bt.phi, bt.psi, bt.cos_iota, ln_mc=torch.log(bt.mc))
    seg = tfsc.segment_layout(gridspec(g), bt)
    store = tfsc.PixelStore.from_complex(dev(pix), dev(u), dev(wm), dtype="f64", layout="layer")
    a = tfsc.bank_statistic_harmonics(gridspec(g), store, bt, seg, HS, _amp_dev(amps), precision="f64")
    c = tfsc.bank_statistic_harmonics(gridspec(g), store, bl, seg, HS, _amp_dev(amps), precision="f64")
    r = rel(c.stat.cpu().numpy(), a.stat.cpu().numpy())
    # exp(ln Mc) may differ from the stored Mc by an ulp: a phase change of up to ~1e-6 rad over a long track
    assert r.max() < 1e-7
    assert torch.equal(c.flags, a.flags)
