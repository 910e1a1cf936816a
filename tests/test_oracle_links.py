"""Pins of the oracle's unequal-arm response (Sec. "Outlook": numerical orbits with varying arm lengths and
point-ahead light times; the response of Sec. "Implementation details" with each link's own light time).

* For a monochromatic wave and a frozen geometry, the time-domain links and delays written out
  (``response.tdi_xyz_td_frozen``) equal the per-tranche transfer times the carrier, to rounding, with six
  different link light times.  A table with the two directions of each arm swapped, or the delays of the
  reverse links, does not match.
* Six equal light times L on a table whose sides are exactly L give the equal-arm transfer of the same table.
* For a chirping source the time-domain form and the transfer agree to the per-tranche approximation's
  2e-3, as for equal arms.
* In the statistic: equal links on an exactly equilateral orbit give the equal-arm statistic; a longer arm
  changes it.
* Second TDI generation: the time-domain combination minus itself delayed by both round trips equals the
  transfer times the carrier for a monochromatic wave; for equal arms it is the first generation times the
  closed form 1 - exp(-8 pi i f L), and for unequal arms the three channels get different factors.
"""
import math

import numpy as np
import pytest
import torch

import tfsc_inputs as ti
from oracle import o2
from oracle import response as rsp
from oracle import track as trk


def _sky_pars():
    return [(0.3, 1.0, 0.4, 0.6), (-0.8, 4.0, 2.2, -0.1), (0.95, 2.5, 1.3, 0.9)]


def _links(seed, spread=0.06):
    rng = np.random.default_rng(seed)
    return rsp.L_S * (1.0 + spread * rng.uniform(-1.0, 1.0, size=6))


def _mono(f, ci):
    ap = (1.0 + ci * ci) / 2.0

    def hfun(tq):
        e = torch.polar(torch.ones_like(tq), 2.0 * math.pi * f * tq)
        return ap * e, torch.complex(torch.zeros_like(tq), -ci * torch.ones_like(tq)) * e

    return hfun


def _equilateral(t0, side):
    """Three spacecraft on an exact equilateral triangle of the given side, in the analytic orbit's plane at
    time t0 (centre and orientation from the analytic positions)."""
    p = rsp.orbits(torch.tensor(t0, dtype=torch.float64))
    c = p.mean(dim=0)
    e1 = p[0] - c
    e1 = e1 / torch.linalg.norm(e1)
    nrm = torch.linalg.cross(p[1] - p[0], p[2] - p[0])
    e2 = torch.linalg.cross(nrm / torch.linalg.norm(nrm), e1)
    rad = side / math.sqrt(3.0)
    return torch.stack([c + rad * (math.cos(b) * e1 + math.sin(b) * e2)
                        for b in (0.0, 2.0 * math.pi / 3.0, 4.0 * math.pi / 3.0)])


@pytest.mark.parametrize("ct,ph,ps,ci", _sky_pars())
@pytest.mark.parametrize("f", [0.004, 0.031, 0.087])
def test_monochromatic_time_domain_is_the_transfer(ct, ph, ps, ci, f):
    pos = rsp.orbits(torch.tensor(4.1e6, dtype=torch.float64))
    links = _links(int(1000 * f) + int(10 * (ct + 1.0)))
    t = torch.linspace(2.0e5, 9.0e5, 7, dtype=torch.float64)
    X, Y, Z = rsp.tdi_xyz_td_frozen(t, _mono(f, ci), ct, ph, ps, pos, links)
    fz = torch.full((1,), f, dtype=torch.float64)
    TX, TY, TZ = rsp.transfer_xyz(torch.zeros(1, dtype=torch.float64), fz, ct, ph, ps, ci, pos[None],
                                  torch.as_tensor(links)[None])
    carrier = torch.polar(torch.ones_like(t), 2.0 * math.pi * f * t)
    for td, T in ((X, TX), (Y, TY), (Z, TZ)):
        ref = T * carrier
        err = float(((td - ref).abs() / ref.abs().max()).max())
        assert err < 1e-9, err


def test_swapped_directions_or_reverse_delays_do_not_match():
    ct, ph, ps, ci = _sky_pars()[0]
    f = 0.031
    pos = rsp.orbits(torch.tensor(4.1e6, dtype=torch.float64))
    links = _links(5)
    t = torch.linspace(2.0e5, 9.0e5, 5, dtype=torch.float64)
    X, _, _ = rsp.tdi_xyz_td_frozen(t, _mono(f, ci), ct, ph, ps, pos, links)
    carrier = torch.polar(torch.ones_like(t), 2.0 * math.pi * f * t)
    fz = torch.full((1,), f, dtype=torch.float64)
    swapped = np.concatenate([links[3:], links[:3]])
    TXs, _, _ = rsp.transfer_xyz(torch.zeros(1, dtype=torch.float64), fz, ct, ph, ps, ci, pos[None],
                                 torch.as_tensor(swapped)[None])
    assert float(((X - TXs * carrier).abs() / X.abs().max()).max()) > 1e-3
    # the delay of link 1 -> 3 taken as that link's own light time (not the path back, 3 -> 1) fails too
    Ls = {sr: float(links[row]) for row, sr in enumerate(rsp.LINK_ROWS)}
    wrong = links.copy()
    wrong[rsp.LINK_ROWS.index((2, 0))] = Ls[(0, 2)]
    TXw, _, _ = rsp.transfer_xyz(torch.zeros(1, dtype=torch.float64), fz, ct, ph, ps, ci, pos[None],
                                 torch.as_tensor(wrong)[None])
    assert float(((X - TXw * carrier).abs() / X.abs().max()).max()) > 1e-3


@pytest.mark.parametrize("ct,ph,ps,ci", _sky_pars())
def test_equal_links_on_an_equilateral_table_are_the_equal_arm_form(ct, ph, ps, ci):
    t = torch.tensor([1.0e6, 7.0e6, 2.2e7], dtype=torch.float64)
    pos = torch.stack([_equilateral(float(x), rsp.L_S) for x in t])
    sides = rsp.link_lengths(pos)
    assert float((sides - rsp.L_S).abs().max()) < 1e-12
    f = torch.tensor([0.006, 0.043, 0.091], dtype=torch.float64)
    eq = rsp.transfer_aet(t, f, ct, ph, ps, ci, pos)
    lk = rsp.transfer_aet(t, f, ct, ph, ps, ci, pos, torch.full((3, 6), rsp.L_S, dtype=torch.float64))
    for a, b in zip(eq, lk):
        assert float(((a - b).abs() / a.abs().max()).max()) < 1e-12


def test_chirp_time_domain_matches_transfer_with_unequal_links():
    ct, ph, ps, ci = _sky_pars()[1]
    tpl = trk.Template(torch.tensor(30.0, dtype=torch.float64), torch.tensor(0.25, dtype=torch.float64),
                       torch.tensor(0.02, dtype=torch.float64))
    ap = (1 + ci * ci) / 2

    def hfun(tq):
        Phi, _, _, A = tpl.at(tq)
        e = torch.polar(torch.ones_like(Phi), Phi)
        return A * ap * e, A * torch.complex(torch.zeros_like(Phi), -ci * torch.ones_like(Phi)) * e

    pos = rsp.orbits(torch.tensor(1.3e7, dtype=torch.float64))
    links = _links(11)
    t = torch.linspace(1e5, 3e7, 40, dtype=torch.float64)
    X, Y, Z = rsp.tdi_xyz_td_frozen(t, hfun, ct, ph, ps, pos, links)
    Phi, f, _, Am = tpl.at(t)
    n = t.shape[0]
    TX, TY, TZ = rsp.transfer_xyz(t, f, ct, ph, ps, ci, pos[None].expand(n, 3, 3),
                                  torch.as_tensor(links)[None].expand(n, 6))
    carrier = Am * torch.polar(torch.ones_like(Phi), Phi)
    for td, T in ((X, TX), (Y, TY), (Z, TZ)):
        ref = T * carrier
        assert float(((td - ref).abs() / ref.abs().max()).max()) < 2e-3


def _statistic_setup():
    g = ti.custom_grid(2, 512, 160, dt=5.0, modulated=True, gapped=True, cfg_id=23)
    pix = ti.pixel_noise((2, g.n_bins, g.n_tranches), cfg_id=23, stream=5)
    from oracle import transform as tf
    _, u, wm = tf.whitening(g.tranche_len, g.dt, 0.1, ti.psd_on_bins(g), ti.tranche_psd_scale(g),
                            ti.tranche_keep(g))
    b = ti.random_bank(8, 23, mc_range=(8.0, 40.0), f0_range=(0.01, 0.05), stream=33)
    t = np.arange(g.n_tranches) * g.tranche_dur
    tab = torch.stack([_equilateral(float(x), rsp.L_S) for x in t]).permute(1, 2, 0).numpy().copy()
    return g, pix, u, wm, b, tab


def test_statistic_with_equal_links_on_an_equilateral_orbit():
    g, pix, u, wm, b, tab = _statistic_setup()
    a = o2.statistic(pix, u, wm, b, g, orbit=tab)
    lk = np.full((6, g.n_tranches), rsp.L_S)
    c = o2.statistic(pix, u, wm, b, g, orbit=tab, links=lk)
    assert np.max(np.abs(c.stat - a.stat) / np.maximum(a.stat, 1.0)) < 1e-11
    # one arm 4% longer in both directions moves the statistic
    lk2 = lk.copy()
    lk2[1] *= 1.04
    lk2[4] *= 1.04
    d = o2.statistic(pix, u, wm, b, g, orbit=tab, links=lk2)
    assert np.max(np.abs(d.stat - a.stat) / np.maximum(a.stat, 1.0)) > 1e-4
    assert np.array_equal(d.flags, a.flags)


@pytest.mark.parametrize("ct,ph,ps,ci", _sky_pars()[:2])
@pytest.mark.parametrize("f", [0.009, 0.052])
def test_second_generation_time_domain_is_the_transfer(ct, ph, ps, ci, f):
    pos = rsp.orbits(torch.tensor(9.3e6, dtype=torch.float64))
    links = _links(int(1000 * f) + 40)
    t = torch.linspace(3.0e5, 8.0e5, 5, dtype=torch.float64)
    X, Y, Z = rsp.tdi_xyz_td_frozen(t, _mono(f, ci), ct, ph, ps, pos, links, generation=2)
    fz = torch.full((1,), f, dtype=torch.float64)
    T2 = rsp.transfer_xyz(torch.zeros(1, dtype=torch.float64), fz, ct, ph, ps, ci, pos[None],
                          torch.as_tensor(links)[None], generation=2)
    T1 = rsp.transfer_xyz(torch.zeros(1, dtype=torch.float64), fz, ct, ph, ps, ci, pos[None],
                          torch.as_tensor(links)[None])
    carrier = torch.polar(torch.ones_like(t), 2.0 * math.pi * f * t)
    ratios = []
    for td, T, T1c in zip((X, Y, Z), T2, T1):
        ref = T * carrier
        assert float(((td - ref).abs() / ref.abs().max()).max()) < 1e-9
        ratios.append(complex(T[0] / T1c[0]))
    # unequal arms: each channel's own factor
    assert abs(ratios[0] - ratios[1]) > 1e-3 and abs(ratios[1] - ratios[2]) > 1e-3


def test_second_generation_with_equal_arms_is_the_common_factor():
    ct, ph, ps, ci = _sky_pars()[2]
    t = torch.tensor([2.0e6, 1.1e7], dtype=torch.float64)
    pos = torch.stack([_equilateral(float(x), rsp.L_S) for x in t])
    f = torch.tensor([0.017, 0.066], dtype=torch.float64)
    lk = torch.full((2, 6), rsp.L_S, dtype=torch.float64)
    one = rsp.transfer_xyz(t, f, ct, ph, ps, ci, pos, lk)
    two = rsp.transfer_xyz(t, f, ct, ph, ps, ci, pos, lk, generation=2)
    factor = 1.0 - torch.polar(torch.ones_like(f), -8.0 * math.pi * f * rsp.L_S)
    for a, b in zip(one, two):
        assert float(((b - factor * a).abs() / b.abs().max()).max()) < 1e-12
