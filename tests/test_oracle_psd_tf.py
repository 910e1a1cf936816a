"""Pins of the oracle's PSD that varies between tranches in a general way (paper Sec. "Search extension to
data with gaps": a time-frequency PSD that differs from tranche to tranche, for locally stationary noise).

The per-pixel path (``transform.transform_tf`` + ``o2.statistic(weight_tf=...)``) is checked against the
separable path it must reduce to, against the exact scaling of Upsilon with the PSD level, and against a
pixel-by-pixel loop that applies 1/sqrt(S_m(f_k)) to data and template by hand.
"""
import numpy as np
import pytest

import tfsc_inputs as ti
from oracle import o2
from oracle import track as trk
from oracle import transform as tf


def _setup(g):
    psd = ti.psd_on_bins(g)
    mu = ti.tranche_psd_scale(g)
    keep = ti.tranche_keep(g)
    x = ti.noise(g)
    b = ti.random_bank(5, 9, mc_range=(15.0, 50.0), f0_range=(0.012, 0.035), stream=23)
    return psd, mu, keep, x, b


def test_separable_psd_reduces_to_the_separable_path(small_grid):
    """S_m(f_k) = mu_m S0(f_k) given pixel by pixel: same pixels and the same statistic as the separable
    whitening with weights u_k w_m.  mu varies with m and S0 with k, so a transposed index fails."""
    g = small_grid
    psd, mu, keep, x, b = _setup(g)
    S = psd[:, None] * mu[None, :]
    assert S.shape == (g.n_bins, g.n_tranches) and g.n_bins != g.n_tranches
    pix, u, wm = tf.transform(x, g, psd, mu, keep, 0.1, "rfft")
    pix_tf, wt = tf.transform_tf(x, g, S, keep, 0.1, "rfft")
    np.testing.assert_allclose(pix_tf, pix, rtol=1e-14, atol=0.0)
    np.testing.assert_allclose(wt, u[:, None] * wm[None, :], rtol=1e-15, atol=0.0)
    lay = trk.Layout(b, g)
    a = o2.statistic(pix, u, wm, b, g, layout=lay)
    c = o2.statistic(pix_tf, None, None, b, g, layout=lay, weight_tf=wt)
    np.testing.assert_allclose(c.stat, a.stat, rtol=1e-12, atol=0.0)
    np.testing.assert_allclose(c.seg_terms, a.seg_terms, rtol=1e-12, atol=1e-300)
    assert np.array_equal(c.flags, a.flags)
    with pytest.raises(ValueError):
        o2.statistic(pix_tf, u, None, b, g, layout=lay, weight_tf=wt)


def test_psd_level_scales_upsilon_inversely(small_grid):
    """S -> 4 S whitens the data and weights the template by 1/2 each: z_n -> z_n / 4, N_n -> N_n / 4,
    so Upsilon -> Upsilon / 4 exactly (a weight applied to one side only would give 1/2 or 1)."""
    g = small_grid
    psd, mu, keep, x, b = _setup(g)
    S = ti.tranche_psd_tf(g)
    lay = trk.Layout(b, g)
    p1, w1 = tf.transform_tf(x, g, S, keep, 0.1, "rfft")
    p4, w4 = tf.transform_tf(x, g, 4.0 * S, keep, 0.1, "rfft")
    r1 = o2.statistic(p1, None, None, b, g, layout=lay, weight_tf=w1)
    r4 = o2.statistic(p4, None, None, b, g, layout=lay, weight_tf=w4)
    assert np.all(r1.stat[r1.stat > 0] > 0)
    np.testing.assert_allclose(r4.stat, r1.stat / 4.0, rtol=1e-12, atol=0.0)


def test_non_separable_psd_matches_a_pixel_loop(small_grid):
    """A drifting spectral tilt (not a product mu_m S0_k): the statistic equals z_n and N_n summed pixel
    by pixel from unit-PSD pixels and unit-weight template pixels, each divided by sqrt(S_m(f_k))."""
    g = small_grid
    psd, mu, keep, x, b = _setup(g)
    S = ti.tranche_psd_tf(g)
    # the tilt really is not separable: log S is not a sum f(k) + g(m)
    L = np.log(S[1:-1])
    resid = L - L.mean(axis=0, keepdims=True) - L.mean(axis=1, keepdims=True) + L.mean()
    assert np.abs(resid).max() > 0.05
    pix_tf, wt = tf.transform_tf(x, g, S, keep, 0.1, "rfft")
    ones_k = np.ones(g.n_bins)
    keep01 = (np.asarray(keep) > 0).astype(np.float64)
    pix_unit, _, _ = tf.transform(x, g, ones_k, np.ones(g.n_tranches), keep, 0.1, "rfft")
    lay = trk.Layout(b, g)
    res = o2.statistic(pix_tf, None, None, b, g, layout=lay, weight_tf=wt)
    for i in range(len(b)):
        if lay.flags[i] & (trk.FLAG_INVALID | trk.FLAG_EMPTY):
            continue
        m, kc, k, valid, Y1 = o2.template_pixels(b.mc[i], b.eta[i], b.f0[i], b.cos_theta[i], b.phi[i], b.psi[i],
                                                 b.cos_iota[i], lay.m_end[i], g, ones_k, keep01)
        m, k, valid, Y1 = m.numpy(), k.numpy(), valid.numpy(), Y1.numpy()
        ns = int(lay.nseg[i])
        z = np.zeros(ns, np.complex128)
        N = np.zeros(ns)
        for a in range(len(m)):
            n = (int(m[a]) * ns) // g.n_tranches
            for jj in range(k.shape[1]):
                if not valid[a, jj]:
                    continue
                kk, mm = int(k[a, jj]), int(m[a])
                r = 1.0 / np.sqrt(S[kk, mm])
                for c in range(g.n_channels):
                    d = pix_unit[c, kk, mm] * r
                    y = Y1[c, a, jj] * r
                    z[n] += np.conj(d) * y
                    N[n] += abs(y) ** 2
        ups = np.where(N > 0, 2.0 * np.abs(z) ** 2 / np.where(N > 0, N, 1.0), 0.0)
        o = lay.seg_offset[i]
        np.testing.assert_allclose(res.seg_terms[o:o + ns], ups, rtol=1e-10, atol=1e-12)
        assert res.stat[i] == pytest.approx(ups.sum(), rel=1e-10)


def test_gradient_with_per_pixel_weights_reduces_to_the_separable_one(small_grid):
    """The oracle gradient through per-pixel weights equals the separable one when S_m(f_k) = mu_m S0(f_k).
    The two weight tables differ by rounding (1/sqrt(S0 mu) against 1/sqrt(S0) / sqrt(mu)), and the float64
    gradient of the literal Fresnel form amplifies rounding to ~1e-7 relative at small beta = fdot dT^2, so
    the bar is 1e-6 with a floor of 1e-3 of the largest component."""
    g = small_grid
    psd, mu, keep, x, b = _setup(g)
    pix, u, wm = tf.transform(x, g, psd, mu, keep, 0.1, "rfft")
    pix_tf, wt = tf.transform_tf(x, g, psd[:, None] * mu[None, :], keep, 0.1, "rfft")
    lay = trk.Layout(b, g)
    for i in range(len(b)):
        if lay.flags[i] & (trk.FLAG_INVALID | trk.FLAG_EMPTY):
            continue
        ga, La = o2.gradient(pix, u, wm, b, g, i, layout=lay)
        gb, Lb = o2.gradient(pix_tf, None, None, b, g, i, layout=lay, weight_tf=wt)
        assert Lb == pytest.approx(La, rel=1e-12)
        err = np.abs(gb - ga) / np.maximum(np.abs(ga), 1e-3 * np.abs(ga).max())
        assert err.max() < 1e-6, (i, err)
