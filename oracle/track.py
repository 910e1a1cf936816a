"""Template track: 2PN TaylorT3 phase, frequency and chirp, plus the
per-template segment layout and track end.

Paper passages followed:
* Sec. "Time-frequency waveform representation": the phase is expanded to
  second order at the *start* of each tranche, t_nm = n T_seg + m dT, with
  f_nm = phi'(t_nm) / 2pi and fdot_nm = phi''(t_nm) / 2pi; A_nm = A(t_nm).
* Sec. "Methods" (timescale hierarchy): segments are non-overlapping and of
  equal length; N_seg is set per template (here from fdot at t = 0).
* Appendix A: a tranche is compact if fdot dT <= 10 delta f.

The paper's own templates are TaylorF2Ecc with chi_eff = 0; its phasing
formulas are not reproduced in the text.  The oracle uses the non-spinning
quasi-circular 2PN TaylorT3 family (Blanchet-Iyer), stated here in
theta = [eta (t_c - t) / (5 M)]^(-1/8):

  Phi(t) = 2 phi_c - (2/eta) theta^-5 [1 + b2 theta^2 + b3 theta^3 + b4 theta^4]
  f(t)   = theta^3 / (8 pi M) [1 + a2 theta^2 + a3 theta^3 + a4 theta^4]
  dtheta/dt = eta theta^9 / (40 M)

with M = Mc eta^(-3/5) in seconds (phi_c = 0).  Readings fixed here:
* f0 = f(t = 0); theta0 solves f(theta0) = f0 by 6 Newton steps from the
  0PN guess, then t_c = 5 M theta0^-8 / eta.
* eta^(1/5) and the 0PN cube root are formed by fixed-count Newton
  iterations so that only +, -, *, / and sqrt decide the integer outputs
  (bin index, track end, N_seg); every operation is written in a fixed
  order, without fused multiply-add, as the formulas above read: the
  divisions by 5M, 8 pi M, 40M and eta are divisions, theta = 1/s with
  s = [eta (t_c - t)/(5M)]^(1/8) by three square roots, and
  theta^-5 = 1/(theta^4 theta).
* N_seg = clamp(2^round(log2(16 (fdot0 / 1.34e-12)^(1/3))), 16, 256),
  evaluated as 16 * 2^n with n the number of thresholds
  fdot0 >= 1.34e-12 * 2^(3i - 3/2), i = 1..4 (ties round up).
* The track ends before the first tranche m where t_m + dT >= t_c, or
  f_m + fdot_m dT >= f_Nyq - 11 delta f, or fdot_m dT > 10 delta f.
* Flags: 1 invalid parameters, 2 empty track, 4 ended by the band or
  compactness condition, 8 ended by the merger condition, 16 every active
  tranche excluded.
"""
from __future__ import annotations

import math

import numpy as np
import torch

MSUN_S = 4.925490947e-6          # G Msun / c^3 [s]
PI = 3.141592653589793
FDOT_REF = 1.34e-12              # Hz/s, reference chirp rate of the N_seg rule

FLAG_INVALID = 1
FLAG_EMPTY = 2
FLAG_BAND_END = 4
FLAG_MERGE_END = 8
FLAG_ALL_EXCLUDED = 16


def _t(x):
    return x if torch.is_tensor(x) else torch.as_tensor(x, dtype=torch.float64)


class _CRSqrt(torch.autograd.Function):
    """Correctly rounded square root (torch's CPU float64 sqrt is not)."""

    @staticmethod
    def forward(ctx, x):
        y = torch.from_numpy(np.ascontiguousarray(np.sqrt(x.detach().numpy()), dtype=np.float64))
        ctx.save_for_backward(y)
        return y

    @staticmethod
    def backward(ctx, g):
        (y,) = ctx.saved_tensors
        return g / (2.0 * y)


def crsqrt(x):
    """IEEE correctly rounded sqrt with autograd (the track's integer outputs depend on it)."""
    return _CRSqrt.apply(_t(x).contiguous())


def pn_coefficients(eta):
    """(a2, a3, a4) of f(theta) and (b2, b3, b4) of Phi(theta)."""
    eta = _t(eta)
    e2 = eta * eta
    a2 = 743.0 / 2688.0 + (11.0 / 32.0) * eta
    a3 = -3.0 * PI / 10.0 + 0.0 * eta
    a4 = (1855099.0 / 14450688.0 + (56975.0 / 258048.0) * eta) + (371.0 / 2048.0) * e2
    b2 = 3715.0 / 8064.0 + (55.0 / 96.0) * eta
    b3 = -3.0 * PI / 4.0 + 0.0 * eta
    b4 = (9275495.0 / 14450688.0 + (284875.0 / 258048.0) * eta) + (1855.0 / 2048.0) * e2
    return a2, a3, a4, b2, b3, b4


def eta_fifth_root(eta):
    """eta^(1/5) by 12 Newton steps on y^5 = eta from y = 1."""
    eta = _t(eta)
    y = torch.ones_like(eta)
    for _ in range(12):
        y4 = (y * y) * (y * y)
        y = (4.0 * y + eta / y4) / 5.0
    return y


def total_mass_s(mc, eta):
    """Total mass M = Mc eta^(-3/5) in seconds."""
    mc, eta = _t(mc), _t(eta)
    y = eta_fifth_root(eta)
    return (mc * MSUN_S) / ((y * y) * y)


class Template:
    """Per-template constants of the T3 track (tensors broadcast over a batch)."""

    def __init__(self, mc, eta, f0):
        self.mc, self.eta, self.f0 = _t(mc), _t(eta), _t(f0)
        self.M = total_mass_s(self.mc, self.eta)
        self.a2, self.a3, self.a4, self.b2, self.b3, self.b4 = pn_coefficients(self.eta)
        self.c8 = (8.0 * PI) * self.M
        self.theta0 = self._solve_theta0()
        th2 = self.theta0 * self.theta0
        th4 = th2 * th2
        th8 = th4 * th4
        self.tc = (5.0 * self.M) / (self.eta * th8)

    def _solve_theta0(self):
        z = self.c8 * self.f0
        y = crsqrt(crsqrt(z))
        for _ in range(10):
            y = (2.0 * y + z / (y * y)) / 3.0
        th = y
        for _ in range(6):
            th2 = th * th
            th3 = th2 * th
            th4 = th2 * th2
            P = ((1.0 + self.a2 * th2) + self.a3 * th3) + self.a4 * th4
            F = th3 * P - z
            dP = ((3.0 + (5.0 * self.a2) * th2) + (6.0 * self.a3) * th3) + (7.0 * self.a4) * th4
            th = th - F / (th2 * dP)
        return th

    def theta(self, t):
        """theta(t) = [eta (t_c - t) / (5 M)]^(-1/8) by three square roots."""
        tau = self.tc - _t(t)
        q = (self.eta * tau) / (5.0 * self.M)
        s = crsqrt(crsqrt(crsqrt(q)))
        return 1.0 / s

    def at(self, t):
        """(Phi, f, fdot, A) at times t (valid for t < t_c)."""
        th = self.theta(t)
        th2 = th * th
        th3 = th2 * th
        th4 = th2 * th2
        Pf = ((1.0 + self.a2 * th2) + self.a3 * th3) + self.a4 * th4
        f = (th3 / self.c8) * Pf
        dPf = ((3.0 + (5.0 * self.a2) * th2) + (6.0 * self.a3) * th3) + (7.0 * self.a4) * th4
        dfdth = (th2 / self.c8) * dPf
        th8 = th4 * th4
        th9 = th8 * th
        dthdt = (self.eta * th9) / (40.0 * self.M)
        fdot = dfdth * dthdt
        Pp = ((1.0 + self.b2 * th2) + self.b3 * th3) + self.b4 * th4
        thm5 = 1.0 / (th4 * th)
        Phi = -((2.0 * thm5) * Pp) / self.eta
        A = torch.pow(f, 2.0 / 3.0)
        return Phi, f, fdot, A


def params_valid(mc, eta, f0, cos_theta, cos_iota) -> np.ndarray:
    mc, eta, f0 = (np.asarray(v, dtype=np.float64) for v in (mc, eta, f0))
    ct, ci = np.asarray(cos_theta, np.float64), np.asarray(cos_iota, np.float64)
    ok = (mc > 0) & (eta >= 0.01) & (eta <= 0.25) & (f0 > 0)
    ok &= (np.abs(ct) <= 1.0) & (np.abs(ci) <= 1.0)
    ok &= np.isfinite(mc) & np.isfinite(eta) & np.isfinite(f0) & np.isfinite(ct) & np.isfinite(ci)
    return ok


def nseg_rule(fdot0) -> np.ndarray:
    """N_seg = 16 * 2^n, n = #{i in 1..4 : fdot0 >= FDOT_REF * 2^(3i-2) * sqrt(2)}."""
    fd = np.asarray(fdot0, dtype=np.float64)
    n = np.zeros(fd.shape, dtype=np.int64)
    r2 = math.sqrt(2.0)
    for i in range(1, 5):
        thr = FDOT_REF * math.ldexp(r2, 3 * i - 2)
        n += (fd >= thr).astype(np.int64)
    return (16 << n).astype(np.int64)


def seg_index(m, nseg, n_tranches):
    """Segment of tranche m when Nt tranches are cut into nseg equal segments."""
    return (np.asarray(m, dtype=np.int64) * int(nseg)) // int(n_tranches)


class Layout:
    """Per-template bookkeeping shared by O1 and O2: constants, N_seg, track end, flags."""

    def __init__(self, bank, grid, nseg_fixed: int | None = None):
        self.grid = grid
        self.n = len(bank.mc)
        self.valid = params_valid(bank.mc, bank.eta, bank.f0, bank.cos_theta, bank.cos_iota)
        # evaluate constants only on valid rows (invalid rows get harmless stand-ins)
        mc = np.where(self.valid, bank.mc, 30.0)
        eta = np.where(self.valid, bank.eta, 0.25)
        f0 = np.where(self.valid, bank.f0, 0.01)
        self.tpl = Template(torch.tensor(mc), torch.tensor(eta), torch.tensor(f0))
        _, _, fdot0, _ = self.tpl.at(torch.zeros(self.n, dtype=torch.float64))
        self.fdot0 = fdot0.numpy()
        fixed = grid.nseg_fixed if nseg_fixed is None else nseg_fixed
        if fixed:
            self.nseg = np.full(self.n, int(fixed), dtype=np.int64)
        else:
            self.nseg = nseg_rule(self.fdot0)
        self.seg_offset = np.zeros(self.n + 1, dtype=np.int64)
        self.seg_offset[1:] = np.cumsum(self.nseg)
        self.m_end = np.zeros(self.n, dtype=np.int64)
        self.flags = np.zeros(self.n, dtype=np.int64)
        dT = float(grid.tranche_dur)
        df = 1.0 / dT
        fnyq = 0.5 / grid.dt
        Nt = grid.n_tranches
        tm = torch.arange(Nt, dtype=torch.float64) * dT
        for i in range(self.n):
            if not self.valid[i]:
                self.flags[i] = FLAG_INVALID
                continue
            tc = float(self.tpl.tc[i])
            merge = (tm + dT) >= tc
            # the track is only evaluated where tau > dT
            safe_t = torch.where(merge, torch.zeros_like(tm), tm)
            sub = Template(self.tpl.mc[i], self.tpl.eta[i], self.tpl.f0[i])
            _, f, fdot, _ = sub.at(safe_t)
            band = (f + fdot * dT) >= (fnyq - 11.0 * df)
            compact = (fdot * dT) > (10.0 * df)
            stop = merge | band | compact
            idx = torch.nonzero(stop)
            if idx.numel() == 0:
                self.m_end[i] = Nt
            else:
                m = int(idx[0])
                self.m_end[i] = m
                self.flags[i] |= FLAG_MERGE_END if bool(merge[m]) else FLAG_BAND_END
            if self.m_end[i] == 0:
                self.flags[i] |= FLAG_EMPTY

    def template(self, i) -> Template:
        return Template(self.tpl.mc[i], self.tpl.eta[i], self.tpl.f0[i])
