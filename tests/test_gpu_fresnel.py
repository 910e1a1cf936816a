"""The accurate Fresnel mode (tfsc_options.fresnel = TFSC_FRESNEL_ACCURATE: the Fresnel integrals themselves in
Eq. (fresnel-ft) instead of the paper's two-branch approximations) through the C ABI, against the oracle with
scipy's Fresnel integrals (``oracle.o2`` with exact_fresnel=True)."""
import functools

import numpy as np
import pytest

import tfsc_inputs as ti
from oracle import o2
from oracle import track as otrk
from oracle import transform as otf

from gpu_common import dev, gridspec, lib, note, rel

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=1)
def _data():
    """Two channels with gaps and modulation; noise plus the bank's first template injected in the pixel domain
    with the exact Fresnel spectrum (SNR 30), so that the Fresnel mode decides its Upsilon."""
    g = ti.custom_grid(2, 512, 400, dt=5.0, modulated=True, gapped=True, cfg_id=23)
    psd, mu, keep = ti.psd_on_bins(g), ti.tranche_psd_scale(g), ti.tranche_keep(g)
    pix, u, wm = otf.transform(ti.noise(g), g, psd, mu, keep, 0.1, "rfft")
    b = ti.random_bank(48, 23, mc_range=(15.0, 60.0), f0_range=(0.008, 0.04), eta=None, stream=43)
    lay = otrk.Layout(b, g)
    m, kc, k, valid, Y = o2.template_pixels(b.mc[0], b.eta[0], b.f0[0], b.cos_theta[0], b.phi[0], b.psi[0],
                                            b.cos_iota[0], lay.m_end[0], g, u, wm, exact_fresnel=True)
    Y = Y.detach().numpy()
    Y *= 30.0 / np.sqrt(2.0 * np.sum(np.abs(Y) ** 2))
    kk = np.clip(k.numpy(), 0, g.n_bins - 1)
    mm = np.broadcast_to(m.numpy()[:, None], kk.shape)
    v = valid.numpy()
    for c in range(2):
        np.add.at(pix[c], (kk[v], mm[v]), Y[c][v])
    exact = o2.statistic(pix, u, wm, b, g, layout=lay, exact_fresnel=True)
    paper = o2.statistic(pix, u, wm, b, g, layout=lay)
    return g, pix, u, wm, b, exact, paper


@pytest.mark.parametrize("dtype,layout,schedule,tol", [("f64", "layer", "wave", 1e-6), ("f64", "tranche", "thread", 1e-6),
                                                       ("f32", "layer_ci", "wave", 1e-4)])
def test_accurate_fresnel_against_the_oracle(dtype, layout, schedule, tol):
    tfsc = lib()
    g, pix, u, wm, b, exact, paper = _data()
    bt = tfsc.BankTensors.from_host(b)
    seg = tfsc.segment_layout(gridspec(g), bt)
    store = tfsc.PixelStore.from_complex(dev(pix), dev(u), dev(wm), dtype=dtype, layout=layout)
    acc = tfsc.bank_statistic(gridspec(g), store, bt, seg, precision=dtype, schedule=schedule, fresnel="accurate")
    pap = tfsc.bank_statistic(gridspec(g), store, bt, seg, precision=dtype, schedule=schedule)
    s, sp = acc.stat.cpu().numpy(), pap.stat.cpu().numpy()
    r = rel(s, exact.stat)
    rp = rel(sp, paper.stat)
    gap = rel(paper.stat, exact.stat).max()
    note(f"accurate Fresnel {dtype} {schedule}: max rel vs exact oracle {r.max():.2e}; paper form vs paper oracle "
         f"{rp.max():.2e}; the two oracles differ by up to {gap:.2e} (injection: paper {paper.stat[0]:.3f}, "
         f"exact {exact.stat[0]:.3f}, GPU accurate {s[0]:.3f})")
    assert r.max() < tol and rp.max() < tol
    # the comparison tells the two forms apart: the paper's forms miss the exact oracle by far more than the
    # accurate mode does
    assert gap > 100 * r.max()
    assert np.array_equal(acc.flags.cpu().numpy(), exact.flags)
