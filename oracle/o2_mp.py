"""O2 for one template in multiple-precision arithmetic (mpmath), with its gradient.

Test infrastructure only.  The same formulas as ``oracle.o2``:
* TaylorT3 track (``oracle.track``), evaluated exactly (theta0 by a root
  finder at full working precision, no fixed-count iterations);
* the tranche spectrum of Eq. (fresnel-ft) with the paper's two-branch
  Fresnel forms (``oracle.fresnel.fresnel_paper``);
* the response of ``oracle.response.transfer_aet`` (A, E and the third channel T);
* Eqs. (overlap-n), (Upsilon-seg) on the given whitened pixels.

The integer structure (track end, bin indices, Fresnel branch of every
argument, N_seg) is taken from the float64 oracle at the template's own
parameters and held fixed, as the gradient definition does.  The gradient is
a central difference at working precision (default 60 digits, step 1e-15),
so its error is far below float64 rounding.  Its purpose is to judge float64
gradients where they lose digits: for small beta = fdot dT^2 the literal
Fresnel form carries phases pi (f - f_k)^2 / fdot of 1e6 rad and more whose
derivatives cancel between terms.  Slow: about a second per hundred
tranches per evaluation.

Every float64 evaluation also carries the rounding of the tranche phase
itself (Phi reaches 1e9 rad, ulp 1e-7 rad), shared bit for bit by all float64
implementations of the track; ``float64_phase`` adds that rounding to the
exact phase so that float64 results can be judged against the rest of the
arithmetic done exactly.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np
import torch

from . import o2
from . import track as trk
from .response import AU_S, L_S, LINKS, YEAR_S

PARAMS = o2.PARAM_NAMES


class _Ctx:
    """Fixed structure and inputs of one template."""

    def __init__(self, pix, u, wm, bank, grid, i, nseg):
        self.grid = grid
        self.dT = float(grid.tranche_dur)
        self.M = grid.tranche_len
        self.Nt = grid.n_tranches
        self.C = grid.n_channels
        b = bank.subset([i])
        lay = trk.Layout(b, grid, nseg_fixed=nseg) if nseg else trk.Layout(b, grid)
        self.m_end = int(lay.m_end[0])
        self.nseg = int(lay.nseg[0])
        self.eta = float(b.eta[0])
        self.ci = float(b.cos_iota[0])
        self.base = dict(mc=float(b.mc[0]), f0=float(b.f0[0]), cos_theta=float(b.cos_theta[0]),
                         phi=float(b.phi[0]), psi=float(b.psi[0]))
        # integer structure from the float64 oracle
        m = torch.arange(self.m_end, dtype=torch.int64)
        tpl = lay.template(0)
        Phi, f, fdot, A = tpl.at(m.to(torch.float64) * self.dT)
        kc, k, valid = o2._bins(f, self.dT, self.M)
        self.k = k.numpy()
        self.valid = valid.numpy()
        # Fresnel branch of every argument (|v| > 6: asymptotic)
        fk = k.to(torch.float64) / self.dT
        zeta = (f[:, None] - fk) / fdot[:, None]
        r = trk.crsqrt(2.0 * fdot)[:, None]
        self.big0 = (torch.abs(r * zeta) > 6.0).numpy()
        self.big1 = (torch.abs(r * (self.dT + zeta)) > 6.0).numpy()
        self.phi64 = Phi.numpy()
        self.delta = None  # per-tranche float64 phase rounding, set by _set_phase_offsets
        self.pix = np.asarray(pix)
        self.u = np.asarray(u, dtype=np.float64)
        self.wm = np.asarray(wm, dtype=np.float64)


def _fresnel(z, big):
    """Paper's C(z), S(z) with the branch given."""
    az = abs(z)
    sg = mp.sign(z)
    arg = mp.pi / 2 * az * az
    c, s = mp.cos(arg), mp.sin(arg)
    if big:
        S = mp.mpf("0.5") - c / (mp.pi * az)
        C = mp.mpf("0.5") + s / (mp.pi * az)
    else:
        fz = (1 + mp.mpf("0.926") * az) / (2 + mp.mpf("1.792") * az + mp.mpf("3.104") * az * az)
        gz = 1 / (2 + mp.mpf("4.142") * az + mp.mpf("3.492") * az * az + mp.mpf("6.670") * az ** 3)
        S = mp.mpf("0.5") - fz * c - gz * s
        C = mp.mpf("0.5") + fz * s - gz * c
    return C * sg, S * sg


def _track(mc, eta, f0):
    """TaylorT3 constants at full precision: returns a function t -> (Phi, f, fdot, A)."""
    eta = mp.mpf(eta)
    M = mc * mp.mpf(trk.MSUN_S) / eta ** (mp.mpf(3) / 5)
    a2 = mp.mpf(743) / 2688 + mp.mpf(11) / 32 * eta
    a3 = -3 * mp.pi / 10
    a4 = mp.mpf(1855099) / 14450688 + mp.mpf(56975) / 258048 * eta + mp.mpf(371) / 2048 * eta ** 2
    b2 = mp.mpf(3715) / 8064 + mp.mpf(55) / 96 * eta
    b3 = -3 * mp.pi / 4
    b4 = mp.mpf(9275495) / 14450688 + mp.mpf(284875) / 258048 * eta + mp.mpf(1855) / 2048 * eta ** 2
    c8 = 8 * mp.pi * M
    z = c8 * f0
    th0 = mp.findroot(lambda th: th ** 3 * (1 + a2 * th ** 2 + a3 * th ** 3 + a4 * th ** 4) - z, mp.cbrt(z))
    tc = 5 * M / (eta * th0 ** 8)

    def at(t):
        th = (eta * (tc - t) / (5 * M)) ** (-mp.mpf(1) / 8)
        Pf = 1 + a2 * th ** 2 + a3 * th ** 3 + a4 * th ** 4
        f = th ** 3 / c8 * Pf
        dPf = 3 + 5 * a2 * th ** 2 + 6 * a3 * th ** 3 + 7 * a4 * th ** 4
        fdot = th ** 2 / c8 * dPf * (eta * th ** 9 / (40 * M))
        Pp = 1 + b2 * th ** 2 + b3 * th ** 3 + b4 * th ** 4
        Phi = -2 * th ** -5 * Pp / eta
        return Phi, f, fdot, f ** (mp.mpf(2) / 3)

    return at


def _orbits(t):
    R = mp.mpf(AU_S)
    e = mp.mpf(L_S) / (2 * mp.sqrt(3) * R)
    a = 2 * mp.pi * t / mp.mpf(YEAR_S)
    out = []
    for i in range(3):
        b = 2 * mp.pi * i / 3
        out.append([R * mp.cos(a) + e * R / 2 * (mp.cos(2 * a - b) - 3 * mp.cos(b)),
                    R * mp.sin(a) + e * R / 2 * (mp.sin(2 * a - b) - 3 * mp.sin(b)),
                    -mp.sqrt(3) * e * R * mp.cos(a - b)])
    return out


def _sky(ct, phi, psi):
    st = mp.sqrt(1 - ct * ct)
    cp, sp = mp.cos(phi), mp.sin(phi)
    k = [-st * cp, -st * sp, -ct]
    u = [ct * cp, ct * sp, -st]
    v = [sp, -cp, mp.mpf(0)]
    return k, u, v, mp.cos(2 * psi), mp.sin(2 * psi)


def _transfer(t, f, sky, ci):
    k, u, v, c2, s2 = sky
    L = mp.mpf(L_S)
    p = _orbits(t)
    ap = (1 + mp.mpf(ci) ** 2) / 2
    G = {}
    for (s, r) in LINKS:
        d = [p[r][x] - p[s][x] for x in range(3)]
        nn = mp.sqrt(sum(x * x for x in d))
        n = [x / nn for x in d]
        dot = lambda a, b: a[0] * b[0] + a[1] * b[1] + a[2] * b[2]
        kn, nu, nv = dot(n, k), dot(n, u), dot(n, v)
        xp0, xx0 = nu * nu - nv * nv, 2 * nu * nv
        xp = c2 * xp0 + s2 * xx0
        xx = -s2 * xp0 + c2 * xx0
        amp = mp.mpc(ap * xp, -mp.mpf(ci) * xx)
        x = mp.pi * f * L * (1 - kn)
        sinc = mp.sin(x) / x if x != 0 else mp.mpf(1)
        kps = dot([p[s][q] + p[r][q] for q in range(3)], k)
        G[(s, r)] = mp.mpc(0, -mp.pi * f * L) * sinc * mp.expj(-mp.pi * f * (L + kps)) * amp
    D = mp.expj(-2 * mp.pi * f * L)
    om = 1 - D * D
    g = lambda s, r: G[(s - 1, r - 1)]
    TX = om * ((g(3, 1) + D * g(1, 3)) - (g(2, 1) + D * g(1, 2)))
    TY = om * ((g(1, 2) + D * g(2, 1)) - (g(3, 2) + D * g(2, 3)))
    TZ = om * ((g(2, 3) + D * g(3, 2)) - (g(1, 3) + D * g(3, 1)))
    return (TZ - TX) / mp.sqrt(2), (TX - 2 * TY + TZ) / mp.sqrt(6), (TX + TY + TZ) / mp.sqrt(3)


def _set_phase_offsets(cx: _Ctx, p0):
    """delta_m = Phi_m(float64 oracle) - Phi_m(exact) at the base point.

    With these added to the exact phase, the objective is the method evaluated exactly except for the
    float64 rounding of the tranche phases (about 1e-7 rad at Phi ~ 1e9 rad), which every float64
    implementation shares because the track is computed in a fixed IEEE order; the offsets are
    constants, so the gradient is still the exact derivative.
    """
    dT = mp.mpf(cx.dT)
    at = _track(mp.e ** p0["ln_mc"], cx.eta, p0["f0"])
    cx.delta = [mp.mpf(float(cx.phi64[m])) - at(m * dT)[0] for m in range(cx.m_end)]


def _objective(cx: _Ctx, p, g_seg):
    """sum_n g_n Upsilon_n at parameters p (dict of mp values; mc given through ln_mc)."""
    dT = mp.mpf(cx.dT)
    at = _track(mp.e ** p["ln_mc"], cx.eta, p["f0"])
    sky = _sky(p["cos_theta"], p["phi"], p["psi"])
    z = [mp.mpc(0)] * cx.nseg
    N = [mp.mpf(0)] * cx.nseg
    for m in range(cx.m_end):
        w = cx.wm[m]
        if w == 0.0:
            continue
        t = m * dT
        Phi, f, fdot, A = at(t)
        if cx.delta is not None:
            Phi = Phi + cx.delta[m]
        T = _transfer(t, f, sky, cx.ci)[: cx.C]
        r = mp.sqrt(2 * fdot)
        sn = (m * cx.nseg) // cx.Nt
        for jj in range(21):
            if not cx.valid[m, jj]:
                continue
            kk = int(cx.k[m, jj])
            fk = mp.mpf(kk) / dT
            zeta = (f - fk) / fdot
            C1, S1 = _fresnel(r * (dT + zeta), cx.big1[m, jj])
            C0, S0 = _fresnel(r * zeta, cx.big0[m, jj])
            h = A / r * mp.expj(Phi - mp.pi * fdot * zeta * zeta) * mp.mpc(C1 - C0, S1 - S0)
            H = h * mp.mpf(cx.u[kk]) * mp.mpf(w)
            for c in range(cx.C):
                Y = T[c] * H
                D = cx.pix[c, kk, m]
                z[sn] += mp.conj(mp.mpc(float(D.real), float(D.imag))) * Y
                N[sn] += abs(Y) ** 2
    tot = mp.mpf(0)
    for n in range(cx.nseg):
        if N[n] > 0:
            tot += mp.mpf(float(g_seg[n])) * 2 * abs(z[n]) ** 2 / N[n]
    return tot


def gradient(pix, u, wm, bank, grid, i: int, g_seg=None, nseg_fixed: int | None = None, dps: int = 60,
             step: float = 1e-15, float64_phase: bool = False):
    """(value, d value / d(ln Mc, f0, cos theta, phi, psi)) of sum_n g_n Upsilon_n for template i.

    Central differences at ``dps`` digits with relative step ``step`` (absolute for the angles).
    float64_phase: add the float64 oracle's per-tranche phase rounding (see _set_phase_offsets).
    """
    with mp.workdps(dps):
        cx = _Ctx(pix, u, wm, bank, grid, i, nseg_fixed)
        gs = np.ones(cx.nseg) if g_seg is None else np.asarray(g_seg, dtype=np.float64)
        p0 = dict(ln_mc=mp.log(mp.mpf(cx.base["mc"])), f0=mp.mpf(cx.base["f0"]),
                  cos_theta=mp.mpf(cx.base["cos_theta"]), phi=mp.mpf(cx.base["phi"]), psi=mp.mpf(cx.base["psi"]))
        if float64_phase:
            _set_phase_offsets(cx, p0)
        val = _objective(cx, p0, gs)
        h = mp.mpf(step)
        grads = []
        for name in PARAMS:
            dh = h * p0["f0"] if name == "f0" else h
            pp, pm = dict(p0), dict(p0)
            pp[name] = p0[name] + dh
            pm[name] = p0[name] - dh
            grads.append(float((_objective(cx, pp, gs) - _objective(cx, pm, gs)) / (2 * dh)))
        return float(val), np.array(grads)


def statistic(pix, u, wm, bank, grid, i: int, nseg_fixed: int | None = None, dps: int = 40,
              float64_phase: bool = False) -> float:
    """Upsilon of template i at ``dps`` digits (optionally with the float64 phase rounding added)."""
    with mp.workdps(dps):
        cx = _Ctx(pix, u, wm, bank, grid, i, nseg_fixed)
        p0 = dict(ln_mc=mp.log(mp.mpf(cx.base["mc"])), f0=mp.mpf(cx.base["f0"]),
                  cos_theta=mp.mpf(cx.base["cos_theta"]), phi=mp.mpf(cx.base["phi"]), psi=mp.mpf(cx.base["psi"]))
        if float64_phase:
            _set_phase_offsets(cx, p0)
        return float(_objective(cx, p0, np.ones(cx.nseg)))

