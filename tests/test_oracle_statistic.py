"""Pins of the oracle statistic (CPU): closed forms, invariants, noise law, end-to-end SNR."""
import math

import numpy as np
import pytest
import torch

import tfsc_inputs as ti
from oracle import o1, o2
from oracle import track as trk
from oracle import transform as tf


def _grid_weights(g, alpha=0.1):
    psd = ti.psd_on_bins(g)
    mu = ti.tranche_psd_scale(g)
    keep = ti.tranche_keep(g)
    _, u, wm = tf.whitening(g.tranche_len, g.dt, alpha, psd, mu, keep)
    return u, wm


def _small_bank(n=6, seed_stream=21):
    b = ti.random_bank(n, 9, mc_range=(15.0, 50.0), f0_range=(0.012, 0.035), stream=seed_stream)
    return b


def _tpl_pixels(b, i, g, u, wm, nseg=None):
    lay = trk.Layout(b.subset([i]), g, nseg_fixed=nseg)
    m, kc, k, valid, Y = o2.template_pixels(b.mc[i], b.eta[i], b.f0[i], b.cos_theta[i], b.phi[i], b.psi[i],
                                            b.cos_iota[i], lay.m_end[0], g, u, wm)
    return lay, m.numpy(), k.numpy(), valid.numpy(), Y.numpy()


def _scatter(g, m, k, valid, Y, scale=1.0):
    pix = np.zeros((g.n_channels, g.n_bins, g.n_tranches), dtype=np.complex128)
    mm = np.broadcast_to(m[:, None], k.shape)
    for c in range(g.n_channels):
        pix[c, k[valid], mm[valid]] += scale * Y[c][valid]
    return pix


def _stat(pix, u, wm, b, g, nseg):
    lay = trk.Layout(b, g, nseg_fixed=nseg)
    return o2.statistic(pix, u, wm, b, g, layout=lay)


def test_single_segment_is_coherent_overlap(small_grid):
    g = small_grid
    u, wm = _grid_weights(g)
    b = _small_bank()
    pix = ti.pixel_noise((g.n_channels, g.n_bins, g.n_tranches))
    res = _stat(pix, u, wm, b, g, 1)
    for i in range(len(b)):
        lay, m, k, valid, Y = _tpl_pixels(b, i, g, u, wm, 1)
        mm = np.broadcast_to(m[:, None], k.shape)
        D = np.stack([pix[c][np.clip(k, 0, g.n_bins - 1), mm] for c in range(g.n_channels)])
        Dv = D[:, valid]
        Yv = Y[:, valid]
        coh = 2 * abs(np.vdot(Dv.ravel(), Yv.ravel())) ** 2 / np.vdot(Yv.ravel(), Yv.ravel()).real
        assert abs(res.stat[i] - coh) <= 1e-12 * max(1.0, coh)


@pytest.mark.parametrize("nseg", [1, 8, 32, 160])
def test_pixel_domain_injection_gives_optimal_snr2(small_grid, nseg):
    g = small_grid
    u, wm = _grid_weights(g)
    b = _small_bank()
    for i in range(3):
        lay, m, k, valid, Y = _tpl_pixels(b, i, g, u, wm, nseg)
        pix = _scatter(g, m, k, valid, Y, scale=0.37 - 0.2j)
        res = _stat(pix, u, wm, b.subset([i]), g, nseg)
        rho2 = 2 * np.sum(np.abs(pix) ** 2)
        assert abs(res.stat[0] - rho2) <= 1e-12 * rho2
        # the per-segment terms are the per-segment optimal SNR^2
        seg = (np.broadcast_to(m[:, None], k.shape)[valid] * nseg) // g.n_tranches
        per = np.zeros(nseg)
        np.add.at(per, seg, 2 * (np.abs(0.37 - 0.2j * 1) ** 2) * np.sum(np.abs(Y[:, valid]) ** 2, axis=0))
        assert np.allclose(res.seg_terms, per, rtol=1e-12, atol=1e-300)


def test_refinement_is_monotone_and_invariances(small_grid):
    g = small_grid
    u, wm = _grid_weights(g)
    b = _small_bank()
    lay, m, k, valid, Y = _tpl_pixels(b, 0, g, u, wm, 1)
    noise = ti.pixel_noise((g.n_channels, g.n_bins, g.n_tranches), stream=12)
    pix = noise + _scatter(g, m, k, valid, Y, scale=1.5 / math.sqrt(np.sum(np.abs(Y) ** 2)))
    one = b.subset([0])
    vals = [_stat(pix, u, wm, one, g, n).stat[0] for n in (1, 2, 4, 8, 16, 32, 160)]
    assert all(vals[i + 1] >= vals[i] * (1 - 1e-13) for i in range(len(vals) - 1))
    # scaling the data scales Upsilon by |c|^2; scaling the template weights changes nothing
    c = 1.7 - 0.4j
    assert abs(_stat(c * pix, u, wm, one, g, 8).stat[0] - abs(c) ** 2 * vals[3]) < 1e-12 * vals[3]
    assert abs(_stat(pix, u * 3.0, wm, one, g, 8).stat[0] - _stat(pix, u, wm, one, g, 8).stat[0]) < 1e-12 * vals[3]
    # an independent phase per segment leaves Upsilon unchanged
    seg = (np.arange(g.n_tranches) * 8) // g.n_tranches
    rot = np.exp(1j * np.array([0.3, 2.0, -1.0, 4.4, 0.1, 5.5, -2.2, 1.1]))[seg]
    assert abs(_stat(pix * rot[None, None, :], u, wm, one, g, 8).stat[0] - vals[3]) < 1e-12 * vals[3]


def test_noise_law_chi_squared(small_grid):
    """For i.i.d. CN(0,1) pixels each non-empty segment term is chi^2 with 2 dof."""
    g = small_grid
    u, wm = _grid_weights(g)
    b = _small_bank()
    nseg = 16
    lay, m, k, valid, Y = _tpl_pixels(b, 1, g, u, wm, nseg)
    mt = torch.as_tensor(m)
    kt, vt, Yt = torch.as_tensor(k), torch.as_tensor(valid), torch.as_tensor(Y)
    rng = np.random.default_rng(99)
    draws = []
    for _ in range(3000):
        pix = (rng.standard_normal((g.n_channels, g.n_bins, g.n_tranches))
               + 1j * rng.standard_normal((g.n_channels, g.n_bins, g.n_tranches))) / math.sqrt(2)
        z, N = o2._segment_sums(torch.as_tensor(pix), mt, kt, vt, Yt, nseg, g.n_tranches)
        draws.append(float(o2._upsilon(z, N).sum()))
        neff = int((N > 0).sum())
    d = np.array(draws)
    n = d.size
    assert abs(d.mean() - 2 * neff) < 4 * math.sqrt(4 * neff / n)
    assert abs(d.var() - 4 * neff) < 4 * math.sqrt((8 * 2 * neff * (2 * neff + 6)) / n) + 0.05 * 4 * neff


@pytest.fixture(scope="module")
def tiny_injection_data():
    g = ti.TINY
    inj = ti.tiny_injection()
    sig = o1.synthesize(inj, 0, g, analytic=False)
    return g, inj, sig


@pytest.mark.parametrize("alpha,lo,hi", [(0.0, 0.97, 1.0), (0.1, 0.95, 0.995)])
def test_noise_free_injection_recovers_snr2(tiny_injection_data, alpha, lo, hi):
    """Exact-parameter template on noise-free time-domain data: Upsilon ~ match^2 rho^2.

    Whitening uses a flat PSD so that rho^2 = 2 sum |D|^2 over all bins is well defined
    (with a PSD null, window leakage into the null dominates any all-bin sum).  With the
    rectangular window the 21 bins hold ~98.5 % of the power; the Tukey(0.1) data window
    concentrates the data's power in the 21 bins but no longer matches the rectangular
    Fresnel template exactly (measured ~0.984).
    """
    g, inj, sig = tiny_injection_data
    flat = np.ones(g.n_bins)
    ones = np.ones(g.n_tranches)
    pix, u, wm = tf.transform(sig, g, flat, ones, np.ones(g.n_tranches, np.uint8), alpha, "rfft")
    rho2 = 2 * np.sum(np.abs(pix[:, 1:-1]) ** 2)
    tb = ti.tiny_bank().subset([256])          # exact-parameter template
    res = o2.statistic(pix, u, wm, tb, g)
    ratio = res.stat[0] / rho2
    assert lo < ratio <= hi


def test_method_matches_definition_on_same_bins(tiny_injection_data):
    """O2 (Fresnel model, transfer per tranche) vs O1 (time-domain template, direct DFT) on the
    same 21-bin support: the statistics of noise-free data agree to the method's match."""
    g, inj, sig = tiny_injection_data
    psd = ti.psd_on_bins(g)
    mu, keep = ti.tranche_psd_scale(g), ti.tranche_keep(g)
    pix, u, wm = tf.transform(sig, g, psd, mu, keep, 0.1, "rfft")
    tb = ti.tiny_bank().subset([256])
    r2 = o2.statistic(pix, u, wm, tb, g)
    lay = trk.Layout(tb, g)
    Y1 = o1.template_pixels(tb, 0, g, u, wm, alpha=0.0)
    mask = o1.bin_mask(g, lay, 0, "21")
    z, N, ups = o1.statistic_from_pixels(pix, Y1, mask, lay.nseg[0], g.n_tranches)
    assert abs(r2.stat[0] / ups.sum() - 1) < 0.01
    # and O1 with all bins recovers at most what the template sees plus the leakage tail
    maskf = o1.bin_mask(g, lay, 0, "full")
    _, _, upsf = o1.statistic_from_pixels(pix, Y1, maskf, lay.nseg[0], g.n_tranches)
    assert upsf.sum() > 0


def test_gaps_remove_their_share_of_snr2(tiny_injection_data):
    g, inj, sig = tiny_injection_data
    gg = ti.custom_grid(1, g.tranche_len, g.n_tranches, dt=g.dt, gapped=True, nseg_fixed=8, cfg_id=g.cfg_id)
    psd = ti.psd_on_bins(g)
    keep_g = ti.tranche_keep(gg)
    assert 0 < keep_g.sum() < gg.n_tranches
    x_gap = sig * ti.sample_keep_mask(gg)[None, :]
    ones = np.ones(g.n_tranches)
    pix_f, u, wm_f = tf.transform(sig, g, psd, ones, np.ones(g.n_tranches, np.uint8), 0.0, "rfft")
    pix_g, _, wm_g = tf.transform(x_gap, gg, psd, ones, keep_g, 0.0, "rfft")
    tb = ti.tiny_bank().subset([256])
    full = o2.statistic(pix_f, u, wm_f, tb, g).stat[0]
    gap = o2.statistic(pix_g, u, wm_g, tb, gg).stat[0]
    power = np.sum(np.abs(pix_f[0]) ** 2, axis=0)
    kept = power[keep_g > 0].sum() / power.sum()
    assert abs(gap / full - kept) < 0.01
