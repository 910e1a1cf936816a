"""Pins of the oracle's caller-supplied orbit (Sec. "Outlook": numerical and generic orbits at no extra cost;
the response of Sec. "Implementation details" evaluated with the table's spacecraft positions).

* The analytic orbit tabulated at the tranche starts gives the same statistic (to the rounding of torch's
  vectorised cosine over arrays of different lengths).
* The analytic orbit is periodic in one year: the table taken one year later gives the same statistic.
* A rigid rotation of the constellation by an angle a about the ecliptic pole, seen by a source at azimuth
  phi + a, is the analytic constellation seen by the source at phi: same statistic to rounding.  A table
  rotated the wrong way, or a transposed table, fails.
* Moving one spacecraft changes the statistic (the table is read).
"""
import math

import numpy as np
import torch

import tfsc_inputs as ti
from oracle import o2
from oracle import response as rsp
from oracle import track as trk


def _setup():
    g = ti.custom_grid(2, 512, 200, dt=5.0, modulated=True, gapped=True, cfg_id=17)
    pix = ti.pixel_noise((2, g.n_bins, g.n_tranches), cfg_id=17, stream=3)
    from oracle import transform as tf
    _, u, wm = tf.whitening(g.tranche_len, g.dt, 0.1, ti.psd_on_bins(g), ti.tranche_psd_scale(g),
                            ti.tranche_keep(g))
    b = ti.random_bank(10, 17, mc_range=(8.0, 40.0), f0_range=(0.01, 0.05), stream=31)
    # plant the first template's own pixels as a signal so that the statistic depends on the response sharply
    lay = trk.Layout(b, g)
    with torch.no_grad():
        m, kc, k, valid, Y = o2.template_pixels(b.mc[0], b.eta[0], b.f0[0], b.cos_theta[0], b.phi[0], b.psi[0],
                                                b.cos_iota[0], lay.m_end[0], g, u, wm)
    kk = np.clip(k.numpy(), 0, g.n_bins - 1)
    mm = np.broadcast_to(m.numpy()[:, None], kk.shape)
    v = valid.numpy()
    for c in range(2):
        np.add.at(pix[c], (kk[v], mm[v]), 3.0 * Y.numpy()[c][v] / np.sqrt(np.sum(np.abs(Y.numpy()) ** 2)))
    return g, pix, u, wm, b


def _table(g, t0=0.0):
    t = torch.arange(g.n_tranches, dtype=torch.float64) * g.tranche_dur + t0
    return rsp.orbits(t).permute(1, 2, 0).numpy().copy()  # [3 spacecraft][3 coords][Nt]


def _rot_z(tab, a):
    c, s = math.cos(a), math.sin(a)
    out = tab.copy()
    out[:, 0, :] = c * tab[:, 0, :] - s * tab[:, 1, :]
    out[:, 1, :] = s * tab[:, 0, :] + c * tab[:, 1, :]
    return out


def test_analytic_table_is_the_analytic_orbit():
    g, pix, u, wm, b = _setup()
    a = o2.statistic(pix, u, wm, b, g)
    t = o2.statistic(pix, u, wm, b, g, orbit=_table(g))
    assert np.max(np.abs(t.stat - a.stat) / np.maximum(a.stat, 1.0)) < 1e-12
    assert np.max(np.abs(t.seg_terms - a.seg_terms) / np.maximum(a.seg_terms, 1.0)) < 1e-12


def test_one_year_later_is_the_same_orbit():
    g, pix, u, wm, b = _setup()
    a = o2.statistic(pix, u, wm, b, g)
    t = o2.statistic(pix, u, wm, b, g, orbit=_table(g, t0=rsp.YEAR_S))
    assert np.max(np.abs(t.stat - a.stat) / np.maximum(a.stat, 1.0)) < 1e-9


def test_rotated_constellation_is_the_rotated_sky():
    g, pix, u, wm, b = _setup()
    ang = 0.83
    a = o2.statistic(pix, u, wm, b, g)
    br = b.subset(np.arange(len(b)))
    br.phi = b.phi + ang
    r = o2.statistic(pix, u, wm, br, g, orbit=_rot_z(_table(g), ang))
    assert np.max(np.abs(r.stat - a.stat) / np.maximum(a.stat, 1.0)) < 1e-10
    assert np.max(np.abs(r.seg_terms - a.seg_terms) / np.maximum(a.seg_terms, 1.0)) < 1e-10
    # the wrong sense of rotation, or a table with spacecraft and coordinates swapped, does not match
    w = o2.statistic(pix, u, wm, br, g, orbit=_rot_z(_table(g), -ang))
    assert np.max(np.abs(w.stat - a.stat) / np.maximum(a.stat, 1.0)) > 1e-3
    x = o2.statistic(pix, u, wm, b, g, orbit=np.ascontiguousarray(np.transpose(_table(g), (1, 0, 2))))
    assert np.max(np.abs(x.stat - a.stat) / np.maximum(a.stat, 1.0)) > 1e-3


def test_moving_one_spacecraft_changes_the_statistic():
    g, pix, u, wm, b = _setup()
    a = o2.statistic(pix, u, wm, b, g)
    tab = _table(g)
    tab[0, 2, :] += 0.5  # spacecraft 0 displaced by 0.5 light-seconds out of the plane
    t = o2.statistic(pix, u, wm, b, g, orbit=tab)
    assert np.max(np.abs(t.stat - a.stat) / np.maximum(a.stat, 1.0)) > 1e-4
