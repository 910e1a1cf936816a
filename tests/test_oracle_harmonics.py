"""Pins of the oracle's multi-harmonic templates (Sec. "Outlook": {A, f, fdot, phi} per harmonic, the Fresnel
expressions applied to each harmonic).

* The dominant harmonic alone (h = 2, a = 1) is the single-harmonic statistic of ``oracle.o2``.
* A pixel-domain injection of a multi-harmonic template recovers its SNR^2 = 2 sum |Y|^2 for every N_seg
  (Cauchy-Schwarz equality), also where the windows of neighbouring harmonics overlap: a cross term dropped
  from the template norm, or added to only one of z and N, breaks it.
* Multiplying every a_h by one complex constant leaves Upsilon unchanged (per-segment phase and scale).
* In unit-variance complex noise each Upsilon_n is chi-squared with 2 degrees of freedom (mean 2 N_seg),
  which fixes the template norm's normalisation with overlapping windows.
* Each harmonic's O2 template matches the time-domain definition (O1: the strain A e^{i (h/2) Phi} through
  the time-domain links and the direct DFT) on its 21 bins, and a multi-harmonic template matches O1 on the
  union of its windows.
"""
import numpy as np
import pytest
import torch

import tfsc_inputs as ti
from oracle import harmonics as oh
from oracle import o1, o2
from oracle import track as trk
from oracle import transform as tf


def _small():
    g = ti.custom_grid(2, 512, 160, dt=5.0, modulated=True, gapped=True, cfg_id=11)
    psd, mu, keep = ti.psd_on_bins(g), ti.tranche_psd_scale(g), ti.tranche_keep(g)
    _, u, wm = tf.whitening(g.tranche_len, g.dt, 0.1, psd, mu, keep)
    return g, u, wm


def _bank(n, f0_range, stream):
    return ti.random_bank(n, 11, mc_range=(8.0, 40.0), f0_range=f0_range, eta=None, stream=stream)


def test_dominant_harmonic_alone_is_the_single_harmonic_statistic():
    g, u, wm = _small()
    pix = ti.pixel_noise((2, g.n_bins, g.n_tranches), cfg_id=11, stream=5)
    b = _bank(12, (0.004, 0.06), 21)
    a = o2.statistic(pix, u, wm, b, g)
    h = oh.statistic(pix, u, wm, b, g, [2], [1.0])
    assert np.array_equal(a.flags, h.flags) and np.array_equal(a.m_end, h.m_end)
    assert np.max(np.abs(h.stat - a.stat) / np.maximum(a.stat, 1.0)) < 1e-12
    assert np.max(np.abs(h.seg_terms - a.seg_terms) / np.maximum(a.seg_terms, 1.0)) < 1e-12


@pytest.mark.parametrize("f0", [0.006, 0.03])
def test_injection_recovers_snr2_with_and_without_overlapping_windows(f0):
    """f0 = 6 mHz: the orbital frequency is 6 bins at dT = 2560 s, so the windows of h = 1, 2, 3 overlap by
    15 bins; f0 = 30 mHz: they are disjoint."""
    g, u, wm = _small()
    b = _bank(1, (f0, f0 * 1.0001), 22)
    hs, amps = [1, 2, 3], np.array([0.3 - 0.2j, 1.0, 0.5j + 0.1])
    Y = oh.template_column_pixels(b, 0, g, u, wm, hs, amps)
    rho2 = 2.0 * np.sum(np.abs(Y[:, 1:-1]) ** 2)
    for nseg in (None, 1, 5):
        gg = g if nseg is None else ti.custom_grid(2, 512, 160, dt=5.0, modulated=True, gapped=True, cfg_id=11,
                                                   nseg_fixed=nseg)
        r = oh.statistic(Y, u, wm, b, gg, hs, amps)
        assert abs(r.stat[0] / rho2 - 1.0) < 1e-12, (nseg, r.stat[0], rho2)
    # the same data against the dominant harmonic alone recovers less (the other harmonics' power is missed)
    r1 = oh.statistic(Y, u, wm, b, g, [2], [1.0])
    assert r1.stat[0] < 0.999 * rho2
    if f0 < 0.01:
        # with overlapping windows, the norm without the cross terms differs from the true one (by ~5e-6 here:
        # the overlap lies in both windows' tails), far above the 1e-12 of the equality checked above
        m, per = oh.harmonic_pixels(b.mc[0], b.eta[0], b.f0[0], b.cos_theta[0], b.phi[0], b.psi[0], b.cos_iota[0],
                                    oh.track_end(b, g, hs)[0][0], g, u, wm, hs, amps)
        separate = sum(float((Yh.abs() ** 2).sum()) for _, _, Yh in per)
        assert abs(separate / (rho2 / 2.0) - 1.0) > 1e-7


def test_common_complex_factor_leaves_upsilon_unchanged():
    g, u, wm = _small()
    pix = ti.pixel_noise((2, g.n_bins, g.n_tranches), cfg_id=11, stream=6)
    b = _bank(6, (0.004, 0.05), 23)
    hs, amps = [1, 2, 3, 4], np.array([0.2, 1.0, 0.4 - 0.3j, 0.1j])
    a = oh.statistic(pix, u, wm, b, g, hs, amps)
    c = oh.statistic(pix, u, wm, b, g, hs, amps * (2.5 * np.exp(1.1j)))
    assert np.max(np.abs(a.seg_terms - c.seg_terms) / np.maximum(a.seg_terms, 1e-3)) < 1e-11


def test_noise_law_with_overlapping_windows():
    """Upsilon over 300 draws of i.i.d. CN(0, 1) pixels for one overlapping three-harmonic template: mean
    2 N_seg and variance 4 N_seg (chi-squared with 2 N_seg degrees of freedom) within 4 sigma."""
    g = ti.custom_grid(1, 256, 48, dt=5.0, cfg_id=12, nseg_fixed=4)
    u, wm = np.ones(g.n_bins), np.ones(g.n_tranches)
    b = _bank(1, (0.012, 0.0121), 24)
    hs, amps = [1, 2, 3], np.array([0.5, 1.0, 0.7j])
    vals = []
    for d in range(300):
        pix = ti.pixel_noise((1, g.n_bins, g.n_tranches), cfg_id=12, stream=100 + d)
        vals.append(oh.statistic(pix, u, wm, b, g, hs, amps).stat[0])
    vals = np.array(vals)
    ns = 4
    assert abs(vals.mean() - 2 * ns) < 4.0 * np.sqrt(4 * ns / vals.size)
    assert abs(vals.var() / (4 * ns) - 1.0) < 0.3


def test_each_harmonic_matches_the_time_domain_definition():
    """O2's pixels of harmonic h (a_h = 1, the others 0) against O1's direct DFT of the analytic strain
    A e^{i (h/2) Phi} through the time-domain links, on the harmonic's 21 bins (rectangular window, flat PSD);
    then a three-harmonic template on the union of its windows."""
    g0 = ti.TINY
    g = ti.custom_grid(2, g0.tranche_len, 240, dt=g0.dt, nseg_fixed=8, cfg_id=g0.cfg_id)
    flat, ones = np.ones(g.n_bins), np.ones(g.n_tranches)
    _, u, wm = tf.whitening(g.tranche_len, g.dt, 0.0, flat, ones, np.ones(g.n_tranches, np.uint8))
    b = ti.tiny_bank().subset([256])
    for hs, amps in (([1], [1.0]), ([3], [1.0]), ([4], [1.0]), ([1, 2, 3], [0.4, 1.0, 0.3 - 0.2j])):
        Y1 = o1.template_pixels(b, 0, g, u, wm, alpha=0.0, harmonics=(hs, amps))
        Y2 = oh.template_column_pixels(b, 0, g, u, wm, hs, amps)
        mask = np.abs(Y2).sum(axis=0) > 0
        for c in range(2):
            a, bb = Y1[c][mask], Y2[c][mask]
            match = abs(np.vdot(a, bb)) / (np.linalg.norm(a) * np.linalg.norm(bb))
            assert match > 0.99, (hs, c, match)
            assert abs(np.linalg.norm(bb) / np.linalg.norm(a) - 1.0) < 0.03, (hs, c)


def test_highest_harmonic_ends_the_track():
    """The band condition applied to the highest harmonic: a template whose dominant harmonic stays in band
    to the end of the span ends earlier with h = 4 in the set, at the tranche where 2 (f + fdot dT) reaches
    f_Nyq - 11 delta f."""
    g, u, wm = _small()
    b = _bank(1, (0.0478, 0.04781), 25)
    m1, f1, _ = oh.track_end(b, g, [2])
    m4, f4, _ = oh.track_end(b, g, [2, 4])
    assert m4[0] < m1[0] and f4[0] & trk.FLAG_BAND_END
    lay = trk.Layout(b, g)
    tpl = lay.template(0)
    dT = g.tranche_dur
    t = torch.tensor([(m4[0] - 1) * dT, m4[0] * dT], dtype=torch.float64)
    _, f, fd, _ = tpl.at(t)
    lim = 0.5 / g.dt - 11.0 / dT
    assert float(2.0 * (f[0] + fd[0] * dT)) < lim <= float(2.0 * (f[1] + fd[1] * dT))
