"""Pins of the oracle's data transform and whitening (CPU)."""
import numpy as np
import pytest

import tfsc_inputs as ti
from oracle import transform as tf


def test_direct_dft_matches_rfft():
    rng = np.random.default_rng(5)
    x = rng.standard_normal(512 * 7)
    a = tf.tranche_dft(x, 512, 0.1, "direct")
    b = tf.tranche_dft(x, 512, 0.1, "rfft")
    assert np.max(np.abs(a - b)) / np.max(np.abs(b)) < 1e-12


def test_parseval_rectangular():
    rng = np.random.default_rng(6)
    M = 256
    x = rng.standard_normal(M)
    X = tf.tranche_dft(x, M, 0.0, "direct")[:, 0]
    lhs = np.sum(x * x)
    rhs = (abs(X[0]) ** 2 + 2 * np.sum(np.abs(X[1:M // 2]) ** 2) + abs(X[M // 2]) ** 2) / M
    assert abs(lhs - rhs) / lhs < 1e-12


def test_on_bin_tone_is_one_bin():
    M, k0 = 512, 37
    j = np.arange(M)
    x = np.cos(2 * np.pi * k0 * j / M + 0.3)
    X = tf.tranche_dft(x, M, 0.0, "direct")[:, 0]
    assert abs(abs(X[k0]) - M / 2) < 1e-9
    X[k0] = 0
    assert np.max(np.abs(X)) < 1e-9


def test_tukey_window_and_w2():
    w = tf.tukey(2048, 0.1)
    assert abs(np.mean(w * w) - (1 - 5 * 0.1 / 8)) < 1e-3   # continuum value 1 - 5 alpha / 8
    assert w[0] == 0.0 and w[1024] == 1.0
    assert np.allclose(w, w[::-1])


@pytest.mark.parametrize("alpha", [0.0, 0.1])
def test_white_noise_pixels_have_unit_variance(alpha):
    g = ti.custom_grid(1, 512, 400, dt=5.0, cfg_id=5)
    sigma2 = 3.0
    x = ti.white_noise(g, sigma=np.sqrt(sigma2))
    S = 2 * g.dt * sigma2 * np.ones(g.n_bins)     # one-sided PSD of white noise
    pix, u, wm = tf.transform(x, g, S, np.ones(g.n_tranches), np.ones(g.n_tranches, np.uint8), alpha, "rfft")
    p2 = np.abs(pix[0, 1:-1]) ** 2
    n = p2.size
    assert abs(p2.mean() - 1) < 4 / np.sqrt(n) * 1.2
    assert np.allclose(u, 1 / np.sqrt(S)) and np.allclose(wm, 1.0)


def test_coloured_noise_whitened_in_band():
    g = ti.custom_grid(1, 512, 600, dt=5.0, cfg_id=5)
    x = ti.noise(g)
    S0 = ti.psd_on_bins(g)
    pix, _, _ = tf.transform(x, g, S0, np.ones(g.n_tranches), np.ones(g.n_tranches, np.uint8), 0.1, "rfft")
    p2 = np.abs(pix[0]) ** 2
    f = np.arange(g.n_bins) / g.tranche_dur
    band = (f > 1e-2) & (f < 4.5e-2)
    # the PSD is smooth there, so whitening by S0 at the bin gives unit variance to ~1 %;
    # below ~10 mHz leakage of the steep red spectrum through the window raises it
    assert abs(p2[band].mean() - 1) < 0.02
    low = (f > 1e-3) & (f < 3e-3)
    assert p2[low].mean() > 1.5


def test_excluded_tranches_and_modulation():
    g = ti.custom_grid(1, 512, 80, dt=5.0)
    x = ti.white_noise(g)
    S = 2 * g.dt * np.ones(g.n_bins)
    mu = np.linspace(0.8, 1.2, g.n_tranches)
    keep = np.ones(g.n_tranches, np.uint8)
    keep[[3, 40]] = 0
    pix, u, wm = tf.transform(x, g, S, mu, keep, 0.1, "direct")
    assert np.all(pix[0][:, [3, 40]] == 0) and wm[3] == 0 and wm[40] == 0
    assert np.allclose(wm[keep > 0], 1 / np.sqrt(mu[keep > 0]))
    ref, _, _ = tf.transform(x, g, S, np.ones(g.n_tranches), np.ones(g.n_tranches, np.uint8), 0.1, "direct")
    m = 10
    assert np.allclose(pix[0][:, m], ref[0][:, m] / np.sqrt(mu[m]), rtol=1e-13)
