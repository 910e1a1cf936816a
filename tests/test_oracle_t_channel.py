"""Pins of the oracle's third TDI channel T = (X + Y + Z) / sqrt 3 (data-model generality beyond the paper's
A and E, whose response model is paper Eq. (tdi2)).

* A, E, T are an orthonormal combination of X, Y, Z: the summed power of the three equals that of X, Y, Z.
* T is the null channel: its response vanishes at low frequency, faster than f^2 relative to A and E.
* The per-tranche transfer of O2 and the time-domain links of O1 give the same T template on the 21 bins.
"""
import math

import numpy as np
import pytest
import torch

import tfsc_inputs as ti
from oracle import o1, o2
from oracle import response as rsp
from oracle import track as trk
from oracle import transform as tf


def _sky():
    c = lambda v: torch.tensor(v, dtype=torch.float64)
    return c(0.3), c(1.0), c(0.4), c(0.6)


def test_aet_is_an_orthonormal_combination_of_xyz():
    t = torch.linspace(0.0, 6.0e7, 7, dtype=torch.float64)
    for f in (3e-4, 4e-3, 2e-2, 6e-2):
        ff = torch.full_like(t, f)
        A, E, T = rsp.transfer_aet(t, ff, *_sky())
        X, Y, Z = rsp.transfer_xyz(t, ff, *_sky())
        pa = A.abs() ** 2 + E.abs() ** 2 + T.abs() ** 2
        px = X.abs() ** 2 + Y.abs() ** 2 + Z.abs() ** 2
        assert torch.allclose(pa, px, rtol=1e-13, atol=0.0)
        # and A, E are the ones the two-channel response returns
        A2, E2 = rsp.transfer_ae(t, ff, *_sky())
        assert torch.equal(A, A2) and torch.equal(E, E2)


def test_t_is_the_null_channel_at_low_frequency():
    t = torch.tensor([1.0e6, 2.0e7, 5.0e7], dtype=torch.float64)

    def ratio(f):
        A, E, T = rsp.transfer_aet(t, torch.full_like(t, f), *_sky())
        return (T.abs() / torch.sqrt(A.abs() ** 2 + E.abs() ** 2)).numpy()

    assert np.all(ratio(1e-4) < 1e-7)
    for f in (1e-4, 2e-4, 4e-4):
        grow = np.log2(ratio(2 * f) / ratio(f))
        assert np.all(grow > 2.0), (f, grow)
    assert np.all(ratio(3e-2) > 1e-2)  # not null at high frequency


@pytest.fixture(scope="module")
def three_channel_injection():
    g0 = ti.TINY
    g = ti.custom_grid(3, g0.tranche_len, g0.n_tranches, dt=g0.dt, nseg_fixed=8, cfg_id=g0.cfg_id)
    inj = ti.tiny_injection()
    sig = o1.synthesize(inj, 0, g, analytic=False)
    return g, inj, sig


def test_o2_t_template_matches_the_time_domain_definition(three_channel_injection):
    """On the 21 bins of each active tranche the O2 template of every channel (T included) matches the O1
    template (time-domain links, direct DFT) to the method's accuracy; T carries ~1% of A's amplitude at
    15 mHz, so its shape is compared through the normalised overlap."""
    g, inj, sig = three_channel_injection
    flat, ones = np.ones(g.n_bins), np.ones(g.n_tranches)
    _, u, wm = tf.whitening(g.tranche_len, g.dt, 0.0, flat, ones, np.ones(g.n_tranches, np.uint8))
    tb = ti.tiny_bank().subset([256])
    lay = trk.Layout(tb, g)
    Y1 = o1.template_pixels(tb, 0, g, u, wm, alpha=0.0)
    m, kc, k, valid, Y2 = o2.template_pixels(tb.mc[0], tb.eta[0], tb.f0[0], tb.cos_theta[0], tb.phi[0], tb.psi[0],
                                             tb.cos_iota[0], lay.m_end[0], g, u, wm)
    m, k, valid, Y2 = m.numpy(), k.numpy(), valid.numpy(), Y2.numpy()
    mm = np.broadcast_to(m[:, None], k.shape)
    amp = []
    for c in range(3):
        a = Y1[c][np.clip(k, 0, g.n_bins - 1), mm][valid]
        b = Y2[c][valid]
        match = abs(np.vdot(a, b)) / (np.linalg.norm(a) * np.linalg.norm(b))
        assert match > 0.99, (c, match)
        assert abs(np.linalg.norm(b) / np.linalg.norm(a) - 1.0) < 0.02, c
        amp.append(np.linalg.norm(b))
    assert 1e-3 < amp[2] / amp[0] < 0.1
