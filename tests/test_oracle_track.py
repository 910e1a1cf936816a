"""Pins of the oracle's TaylorT3 track, N_seg rule and track end (CPU)."""
import math

import numpy as np
import pytest
import sympy as sp
import torch

import tfsc_inputs as ti
from oracle import track as trk


def _derive_t3_coefficients():
    """2PN TaylorT3 coefficients from the energy-balance equation, in exact arithmetic.

    E(v) and the flux F(v) are the standard non-spinning 2PN expressions
    (Blanchet's Living Review); dt/dv = -E'(v)/F(v) (units of total mass),
    theta^-8 = eta (t_c - t) / 5, f = v^3 / pi, Phi = 2 int v^3 dt.
    Returns (a2, a3, a4, b2, b3, b4) as sympy expressions in eta.
    """
    v, th, eta = sp.symbols("v theta eta", positive=True)
    R = sp.Rational
    E = -R(1, 2) * eta * v ** 2 * (1 - (R(3, 4) + eta / 12) * v ** 2
                                   - (R(27, 8) - R(19, 8) * eta + eta ** 2 / 24) * v ** 4)
    F = R(32, 5) * eta ** 2 * v ** 10 * (1 - (R(1247, 336) + R(35, 12) * eta) * v ** 2 + 4 * sp.pi * v ** 3
                                         - (R(44711, 9072) - R(9271, 504) * eta - R(65, 18) * eta ** 2) * v ** 4)
    ratio = sp.series(sp.simplify(-sp.diff(E, v) / F * v ** 9 * R(32, 5) * eta), v, 0, 5).removeO()
    r = [sp.expand(ratio).coeff(v, k) for k in range(5)]
    # t_c - t = (5/(32 eta)) sum_k r_k v^(k-8)/(8-k);  phi_orb = -(1/(32 eta)) sum_k 5 r_k v^(k-5)/(5-k) (k != 5)
    T = sum(R(5, 32) / eta * r[k] * v ** (k - 8) / (8 - k) for k in range(5))
    phi = -sum(R(5, 32) / eta * r[k] * v ** (k - 5) / (5 - k) for k in range(5))
    # theta(v) = (eta T / 5)^(-1/8) = 2 v (1 + ...)^(-1/8); revert to v(theta)
    c = sp.symbols("c2 c3 c4")
    v_of_th = th / 2 * (1 + c[0] * th ** 2 + c[1] * th ** 3 + c[2] * th ** 4)
    x = sp.expand(eta * T / 5 * v ** 8 * 256)  # = 1 + O(v^2)
    theta_series = 2 * v * sp.series(x ** R(-1, 8), v, 0, 5).removeO()
    eq = sp.series(theta_series.subs(v, v_of_th) - th, th, 0, 6).removeO()
    sol = sp.solve([sp.expand(eq).coeff(th, k) for k in (3, 4, 5)], c, dict=True)[0]
    v_th = v_of_th.subs(sol)
    fser = sp.expand(sp.series((v_th ** 3 / sp.pi) * 8 * sp.pi / th ** 3, th, 0, 5).removeO())
    a = [sp.simplify(fser.coeff(th, k)) for k in (2, 3, 4)]
    Phi = 2 * phi.subs(v, v_th)
    pser = sp.expand(sp.series(Phi * th ** 5 * (-eta / 2), th, 0, 5).removeO())
    b = [sp.simplify(pser.coeff(th, k)) for k in (2, 3, 4)]
    return a, b, eta


def test_t3_coefficients_follow_from_energy_balance():
    a, b, eta_s = _derive_t3_coefficients()
    for eta in (0.25, 0.2, 0.1):
        ours = trk.pn_coefficients(torch.tensor(eta, dtype=torch.float64))
        ref = [float(x.subs(eta_s, eta)) for x in a + b]
        for o, r in zip(ours, ref):
            assert abs(float(o) - r) <= 1e-14 * max(1.0, abs(r)), (o, r)


def _tpl(mc=30.0, eta=0.25, f0=0.015):
    return trk.Template(torch.tensor(mc, dtype=torch.float64), torch.tensor(eta, dtype=torch.float64),
                        torch.tensor(f0, dtype=torch.float64))


@pytest.mark.parametrize("mc,eta,f0", [(30.0, 0.25, 0.015), (7.0, 0.16, 0.028), (90.0, 0.22, 0.004)])
def test_frequency_is_phase_derivative(mc, eta, f0):
    T = _tpl(mc, eta, f0)
    tc = float(T.tc)
    for t in (0.0, 0.3 * tc, 0.9 * tc):
        def d(fun, h):
            a = fun(torch.tensor(t + h, dtype=torch.float64))
            b = fun(torch.tensor(t - h, dtype=torch.float64))
            return (float(a) - float(b)) / (2 * h)
        h = 400.0
        Phi = lambda tt: T.at(tt)[0]
        fref = (4 * d(Phi, h / 2) - d(Phi, h)) / 3 / (2 * math.pi)
        _, f, fdot, A = T.at(torch.tensor(t, dtype=torch.float64))
        assert abs(float(f) - fref) / float(f) < 1e-8
        fun_f = lambda tt: T.at(tt)[1]
        fdref = (4 * d(fun_f, h / 2) - d(fun_f, h)) / 3
        assert abs(float(fdot) - fdref) / float(fdot) < 1e-7
        assert abs(float(A) - float(f) ** (2 / 3)) < 1e-15


@pytest.mark.parametrize("mc,eta,f0", [(30.0, 0.25, 0.015), (5.0, 0.1, 0.002), (100.0, 0.25, 0.09)])
def test_theta0_solves_f0(mc, eta, f0):
    T = _tpl(mc, eta, f0)
    _, f, _, _ = T.at(torch.tensor(0.0, dtype=torch.float64))
    assert abs(float(f) - f0) / f0 < 4e-16
    y = trk.eta_fifth_root(torch.tensor(eta, dtype=torch.float64))
    assert abs(float(y) - eta ** 0.2) < 1e-15


def test_newtonian_chirp_closed_form():
    # leading (0PN) order: f = (1/(8 pi M)) theta^3 with theta^-8 = eta (tc - t)/(5M) is the
    # textbook chirp f = (1/pi) (5/256)^(3/8) Mc^(-5/8) (tc - t)^(-3/8); the 2PN factor is ~1 + a2 theta^2
    T = _tpl(30.0, 0.25, 0.015)
    Mc = 30.0 * trk.MSUN_S
    for frac in (0.0, 0.5):
        t = frac * float(T.tc)
        _, f, _, _ = T.at(torch.tensor(t, dtype=torch.float64))
        f0pn = (1 / math.pi) * (5 / 256) ** (3 / 8) * Mc ** (-5 / 8) * (float(T.tc) - t) ** (-3 / 8)
        th = float(T.theta(torch.tensor(t, dtype=torch.float64)))
        a2 = 743 / 2688 + 11 / 32 * 0.25
        assert abs(float(f) / f0pn - 1 - a2 * th * th) < 5 * th ** 3


def test_t3_agrees_with_energy_balance_ode():
    """T3 vs direct integration of dv/dt = -F/E' (2PN; the two differ at 2.5PN)."""
    from scipy.integrate import solve_ivp
    eta, mc, f0 = 0.25, 60.0, 0.02
    T = _tpl(mc, eta, f0)
    M = float(T.M)

    def rhs(t, y):
        v = y[0]
        dE = -eta * v * (1 - 2 * (3 / 4 + eta / 12) * v ** 2 - 3 * (27 / 8 - 19 * eta / 8 + eta ** 2 / 24) * v ** 4)
        F = 32 / 5 * eta ** 2 * v ** 10 * (1 - (1247 / 336 + 35 * eta / 12) * v ** 2 + 4 * math.pi * v ** 3
                                          - (44711 / 9072 - 9271 * eta / 504 - 65 * eta ** 2 / 18) * v ** 4)
        return [-F / dE / M]

    v0 = (math.pi * M * f0) ** (1 / 3)
    t1 = 0.7 * float(T.tc)
    sol = solve_ivp(rhs, (0, t1), [v0], rtol=1e-12, atol=1e-16, dense_output=True)
    for t in np.linspace(0, t1, 5)[1:]:
        v = sol.sol(t)[0]
        f_ode = v ** 3 / (math.pi * M)
        _, f, _, _ = T.at(torch.tensor(t, dtype=torch.float64))
        assert abs(float(f) / f_ode - 1) < 2e-6 * max(1.0, (v / v0) ** 5 * 10)


def test_nseg_rule_matches_log_form():
    rng = np.random.default_rng(3)
    fd = 10 ** rng.uniform(-13, -7, 200000)
    ours = trk.nseg_rule(fd)
    direct = np.clip(2 ** np.round(np.log2(16 * (fd / trk.FDOT_REF) ** (1 / 3))), 16, 256).astype(np.int64)
    # away from the rounding ties the two forms agree exactly
    y = np.log2(16 * (fd / trk.FDOT_REF) ** (1 / 3))
    far = np.abs(y - np.floor(y) - 0.5) > 1e-9
    assert np.array_equal(ours[far], direct[far])
    thr = [trk.FDOT_REF * 2 ** (3 * i - 1.5) for i in range(1, 5)]
    assert list(trk.nseg_rule(np.array(thr))) == [32, 64, 128, 256]
    assert list(trk.nseg_rule(np.nextafter(np.array(thr), 0))) == [16, 32, 64, 128]


def test_track_end_brute_force():
    g = ti.custom_grid(1, 512, 4000, dt=5.0)
    b = ti.random_bank(40, 9, mc_range=(40.0, 100.0), f0_range=(0.02, 0.06))
    lay = trk.Layout(b, g)
    dT, df, fnyq = g.tranche_dur, 1 / g.tranche_dur, 0.5 / g.dt
    ended = 0
    for i in range(len(b)):
        T = lay.template(i)
        m_first = None
        for m in range(g.n_tranches):
            tm = m * dT
            if tm + dT >= float(T.tc):
                m_first = m
                break
            _, f, fd, _ = T.at(torch.tensor(tm, dtype=torch.float64))
            f, fd = float(f), float(fd)
            if f + fd * dT >= fnyq - 11 * df or fd * dT > 10 * df:
                m_first = m
                break
        expect = g.n_tranches if m_first is None else m_first
        assert lay.m_end[i] == expect
        ended += m_first is not None
    assert ended > 5  # the sample exercises the track-end rule


def test_layout_offsets_and_flags():
    g = ti.custom_grid(1, 512, 300)
    b = ti.random_bank(30, 9)
    b.mc[0] = -1.0
    b.eta[1] = 0.3
    b.f0[2] = 0.2          # above Nyquist: empty track
    lay = trk.Layout(b, g)
    assert lay.flags[0] == trk.FLAG_INVALID and lay.flags[1] == trk.FLAG_INVALID
    assert lay.flags[2] & trk.FLAG_EMPTY and lay.m_end[2] == 0
    assert np.array_equal(np.diff(lay.seg_offset), lay.nseg)
    assert set(np.unique(lay.nseg)) <= {16, 32, 64, 128, 256}
