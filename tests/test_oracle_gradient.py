"""Pin of the oracle gradient: autograd of O2 vs Richardson central differences of O2 (CPU)."""
import math

import numpy as np
import pytest
import torch

import tfsc_inputs as ti
from oracle import o2
from oracle import track as trk
from oracle import transform as tf


def _signature(b, g):
    lay = trk.Layout(b, g)
    T = lay.template(0)
    tm = torch.arange(int(lay.m_end[0]), dtype=torch.float64) * g.tranche_dur
    _, f, fdot, _ = T.at(tm)
    kc = torch.ceil(f * g.tranche_dur).numpy()
    # Fresnel branch of every bin edge
    j = np.arange(-10, 11)
    fk = (kc[:, None] + j[None, :]) / g.tranche_dur
    zeta = (f.numpy()[:, None] - fk) / fdot.numpy()[:, None]
    r = np.sqrt(2 * fdot.numpy())[:, None]
    br = np.concatenate([np.abs(r * zeta) > 6, np.abs(r * (g.tranche_dur + zeta)) > 6], axis=1)
    return (int(lay.m_end[0]), int(lay.nseg[0]), kc.tobytes(), br.tobytes())


@pytest.fixture(scope="module")
def setup():
    g = ti.custom_grid(2, 512, 240, dt=5.0, modulated=True, gapped=True, nseg_fixed=8)
    psd = ti.psd_on_bins(g)
    mu, keep = ti.tranche_psd_scale(g), ti.tranche_keep(g)
    _, u, wm = tf.whitening(g.tranche_len, g.dt, 0.1, psd, mu, keep)
    b = ti.random_bank(4, 9, mc_range=(20.0, 40.0), f0_range=(0.014, 0.02), stream=31)
    # data: noise plus the first template (pixel domain) so the statistic has a peak nearby
    lay = trk.Layout(b.subset([0]), g)
    m, kc, k, valid, Y = o2.template_pixels(b.mc[0], b.eta[0], b.f0[0], b.cos_theta[0], b.phi[0], b.psi[0],
                                            b.cos_iota[0], lay.m_end[0], g, u, wm)
    m, k, valid, Y = m.numpy(), k.numpy(), valid.numpy(), Y.numpy()
    pix = ti.pixel_noise((2, g.n_bins, g.n_tranches), stream=41)
    mm = np.broadcast_to(m[:, None], k.shape)
    sc = 4.0 / math.sqrt(np.sum(np.abs(Y) ** 2))
    for c in range(2):
        pix[c, k[valid], mm[valid]] += sc * Y[c][valid]
    # evaluate the gradient slightly off the injected parameters
    b.f0[0] *= 1 + 2e-7
    b.mc[0] *= 1 - 1e-6
    return g, u, wm, b, pix


@pytest.mark.parametrize("i", [0, 1, 2])
def test_autograd_matches_richardson(setup, i):
    """Three-level Richardson extrapolation of central differences of the O2 forward.

    The forward's own rounding floor is set by the float64 phase (|Phi| ~ 1e7 rad carries
    ~3e-9 rad per tranche), so chirp-parameter steps must stay large and the comparison is
    at 2e-4; the sky and polarisation angles agree to 1e-6.
    """
    g, u, wm, b, pix = setup
    grad, val = o2.gradient(pix, u, wm, b, g, i)
    base, _ = o2.forward_single(pix, u, wm, b, g, i)
    assert abs(val - base) < 1e-12 * max(1.0, base)
    x0 = {"ln_mc": math.log(b.mc[i]), "f0": b.f0[i], "cos_theta": b.cos_theta[i], "phi": b.phi[i], "psi": b.psi[i]}
    steps = {"ln_mc": 4e-4, "f0": 1e-5 * b.f0[i], "cos_theta": 4e-5, "phi": 4e-5, "psi": 4e-5}
    tol = {"ln_mc": 2e-4, "f0": 2e-4, "cos_theta": 1e-6, "phi": 1e-6, "psi": 1e-6}
    sig0 = _signature(b.subset([i]), g)
    checked = 0
    for p_idx, name in enumerate(o2.PARAM_NAMES):
        h = steps[name]
        cd = []
        ok = True
        for hh in (h, h / 2, h / 4):
            vals = []
            for s in (hh, -hh):
                v, _ = o2.forward_single(pix, u, wm, b, g, i, {name: x0[name] + s})
                bb = b.subset([i])
                if name == "ln_mc":
                    bb.mc = np.array([math.exp(x0[name] + s)])
                else:
                    setattr(bb, name, np.array([x0[name] + s]))
                ok &= _signature(bb, g) == sig0
                vals.append(v)
            cd.append((vals[0] - vals[1]) / (2 * hh))
        if not ok:
            continue
        r1 = [(4 * cd[1] - cd[0]) / 3, (4 * cd[2] - cd[1]) / 3]
        rich = (16 * r1[1] - r1[0]) / 15
        ref_scale = max(abs(rich), 1e-2 * abs(base) / (abs(x0[name]) + 1.0))
        assert abs(grad[p_idx] - rich) <= tol[name] * ref_scale, (name, grad[p_idx], rich)
        checked += 1
    assert checked >= 4
