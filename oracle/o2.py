"""O2: the paper's method, written literally, in float64 (torch CPU).

Paper passages followed:
* Eq. (Upsilon-seg) with Eq. (overlap-n): per segment the phase-maximised
  overlap squared over the template norm, summed over segments.
* Eqs. (inner-segment-tf), (inner-tranche-tf): segment inner products are
  sums of tranche inner products; each tranche contributes the transfer
  function T_alpha(f_nm) times the sum over N_F bins of conj(d) h / S.
* Eq. (fresnel-ft) and the Fresnel branches for the tranche spectrum.
* N_F = 21 bins centred on the bin just above f_nm.

Normalisation (a reading; a constant factor changes no ranking): data
pixels D are whitened to unit variance (``oracle.transform``), the template
pixels are Y_cmk = T_c(t_m, f_m) h~_m(f_k) u_k w_m, and with
z_n = sum conj(D) Y and N_n = sum |Y|^2 over the channels, tranches of
segment n and bins of each tranche, Upsilon_n = 2 |z_n|^2 / N_n
(0 when N_n = 0) and Upsilon = sum_n Upsilon_n.  For pure unit-variance
noise each Upsilon_n is chi-squared with 2 degrees of freedom; for D = Y it
equals 2 sum |Y|^2, the optimal SNR^2.

Bins: k_c = ceil(f_m dT) and k = k_c - 10 .. k_c + 10, keeping 1 <= k <= M/2 - 1.
"""
from __future__ import annotations

import numpy as np
import torch

from . import track as trk
from .fresnel import tranche_spectrum
from .response import transfer_aet

NF_HALF = 10
PARAM_NAMES = ("ln_mc", "f0", "cos_theta", "phi", "psi")


def _bins(f_m: torch.Tensor, dT: float, M: int):
    with torch.no_grad():
        kc = torch.ceil(f_m * dT).to(torch.int64)
    j = torch.arange(-NF_HALF, NF_HALF + 1, dtype=torch.int64)
    k = kc[:, None] + j[None, :]
    valid = (k >= 1) & (k <= M // 2 - 1)
    return kc, k, valid


def template_pixels(mc, eta, f0, cos_theta, phi, psi, cos_iota, m_end: int, grid, u, wm,
                    exact_fresnel: bool = False, weight_tf=None, orbit=None, links=None, generation: int = 1):
    """Whitened template pixels of one template on its active tranches.

    Parameters may be 0-d tensors carrying autograd.  Returns (m, kc, k, valid, Y)
    with Y[C, n_m, 21] complex (zero on invalid bins and excluded tranches).
    weight_tf: optional per-pixel weights [K][Nt] (1/sqrt(S_m(f_k)), 0 on excluded
    tranches) for a PSD that varies between tranches in a general way; u and wm
    are then not used.
    orbit: optional spacecraft positions [3][3][Nt] at the tranche starts (light-seconds), the caller's orbit
    in place of the analytic one.
    links: optional link light times [6][Nt] at the tranche starts (light-seconds, rows as
    ``response.LINK_ROWS``): the unequal-arm response in place of the equal-arm one; ``generation`` 2 forms
    it in the second TDI generation.
    """
    dT = float(grid.tranche_dur)
    M = grid.tranche_len
    m = torch.arange(int(m_end), dtype=torch.int64)
    tm = m.to(torch.float64) * dT
    tpl = trk.Template(mc, eta, f0)
    Phi, f, fdot, A = tpl.at(tm)
    kc, k, valid = _bins(f, dT, M)
    fk = k.to(torch.float64) / dT
    h = tranche_spectrum(Phi[:, None], f[:, None], fdot[:, None], A[:, None], fk, dT, exact=exact_fresnel)
    pos = None
    if orbit is not None:
        pos = torch.as_tensor(np.asarray(orbit), dtype=torch.float64)[:, :, m].permute(2, 0, 1)
    lk = None
    if links is not None:
        lk = torch.as_tensor(np.asarray(links), dtype=torch.float64)[:, m].T
    T = list(transfer_aet(tm, f, cos_theta, phi, psi, cos_iota, pos, lk, generation))[: grid.n_channels]
    if weight_tf is not None:
        wt = torch.as_tensor(np.asarray(weight_tf), dtype=torch.float64)
        wkm = wt[k.clamp(0, M // 2), m[:, None]]
        weight = torch.where(valid, wkm, torch.zeros_like(wkm))
    else:
        uk = torch.as_tensor(np.asarray(u), dtype=torch.float64)[k.clamp(0, M // 2)]
        w = torch.as_tensor(np.asarray(wm), dtype=torch.float64)[m]
        weight = torch.where(valid, uk, torch.zeros_like(uk)) * w[:, None]
    Y = torch.stack([Tc[:, None] * h * weight for Tc in T], dim=0)
    return m, kc, k, valid, Y


def _segment_sums(pix_t: torch.Tensor, m, k, valid, Y, nseg: int, Nt: int):
    C = Y.shape[0]
    kk = k.clamp(0, pix_t.shape[1] - 1)
    D = torch.stack([pix_t[c][kk, m[:, None]] for c in range(C)], dim=0)
    D = torch.where(valid[None], D, torch.zeros_like(D))
    zm = (torch.conj(D) * Y).sum(dim=(0, 2))
    Nm = (Y.real * Y.real + Y.imag * Y.imag).sum(dim=(0, 2))
    seg = (m * int(nseg)) // int(Nt)
    z = torch.zeros(int(nseg), dtype=torch.complex128).index_add(0, seg, zm)
    N = torch.zeros(int(nseg), dtype=torch.float64).index_add(0, seg, Nm)
    return z, N


def _upsilon(z, N):
    zz = z.real * z.real + z.imag * z.imag
    safe = torch.where(N > 0, N, torch.ones_like(N))
    return torch.where(N > 0, 2.0 * zz / safe, torch.zeros_like(N))


class Result:
    def __init__(self, n, seg_offset):
        self.stat = np.zeros(n)
        self.seg_offset = seg_offset
        self.seg_terms = np.zeros(int(seg_offset[-1]))
        self.seg_z = np.zeros(int(seg_offset[-1]), dtype=np.complex128)
        self.seg_N = np.zeros(int(seg_offset[-1]))
        self.flags = np.zeros(n, dtype=np.int64)
        self.m_end = np.zeros(n, dtype=np.int64)
        self.nseg = np.zeros(n, dtype=np.int64)


def statistic(pix, u, wm, bank, grid, layout: trk.Layout | None = None, exact_fresnel: bool = False,
              idx=None, weight_tf=None, orbit=None, links=None, generation: int = 1) -> Result:
    """Upsilon and its per-segment terms for every template of ``bank``.

    pix: complex [C][K][Nt] whitened data pixels (numpy), u: [K], wm: [Nt].
    idx: optional subset of template indices (others are left at zero).
    weight_tf: optional per-pixel template weights [K][Nt] in place of u_k w_m
    (``transform.transform_tf``); u and wm must then be None.
    orbit: optional spacecraft positions [3][3][Nt] at the tranche starts (a caller's orbit).
    links: optional link light times [6][Nt] at the tranche starts (unequal arms); generation: TDI 1 or 2.
    """
    if weight_tf is not None and (u is not None or wm is not None):
        raise ValueError("give either (u, wm) or weight_tf")
    if layout is None:
        layout = trk.Layout(bank, grid)
    res = Result(layout.n, layout.seg_offset)
    res.m_end[:] = layout.m_end
    res.nseg[:] = layout.nseg
    res.flags[:] = layout.flags
    pix_t = torch.as_tensor(np.asarray(pix, dtype=np.complex128))
    rows = range(layout.n) if idx is None else idx
    with torch.no_grad():
        for i in rows:
            if layout.flags[i] & (trk.FLAG_INVALID | trk.FLAG_EMPTY):
                continue
            m, kc, k, valid, Y = template_pixels(
                bank.mc[i], bank.eta[i], bank.f0[i], bank.cos_theta[i], bank.phi[i], bank.psi[i],
                bank.cos_iota[i], layout.m_end[i], grid, u, wm, exact_fresnel, weight_tf, orbit, links,
                generation)
            z, N = _segment_sums(pix_t, m, k, valid, Y, layout.nseg[i], grid.n_tranches)
            ups = _upsilon(z, N)
            o = layout.seg_offset[i]
            res.seg_terms[o:o + layout.nseg[i]] = ups.numpy()
            res.seg_z[o:o + layout.nseg[i]] = z.numpy()
            res.seg_N[o:o + layout.nseg[i]] = N.numpy()
            res.stat[i] = float(ups.sum())
            if not bool((N > 0).any()):
                res.flags[i] |= trk.FLAG_ALL_EXCLUDED
    return res


def gradient(pix, u, wm, bank, grid, i: int, g_seg=None, layout: trk.Layout | None = None, weight_tf=None):
    """d(sum_n g_n Upsilon_n)/d(ln Mc, f0, cos theta, phi, psi) for template i (float64 autograd).

    g_seg defaults to all ones (the gradient of Upsilon).  The integer
    structure (bins, branches, track end, N_seg) is held fixed at the
    template's own values; the derivative is the almost-everywhere one.
    """
    if layout is None:
        layout = trk.Layout(bank.subset([i]), grid)
        li = 0
    else:
        li = i
    if layout.flags[li] & (trk.FLAG_INVALID | trk.FLAG_EMPTY):
        return np.zeros(5), 0.0
    pix_t = torch.as_tensor(np.asarray(pix, dtype=np.complex128))
    ln_mc = torch.tensor(float(np.log(bank.mc[i])), dtype=torch.float64, requires_grad=True)
    f0 = torch.tensor(float(bank.f0[i]), dtype=torch.float64, requires_grad=True)
    ct = torch.tensor(float(bank.cos_theta[i]), dtype=torch.float64, requires_grad=True)
    ph = torch.tensor(float(bank.phi[i]), dtype=torch.float64, requires_grad=True)
    ps = torch.tensor(float(bank.psi[i]), dtype=torch.float64, requires_grad=True)
    # value-exact chirp mass: mc * exp(0) with d mc / d ln_mc = mc
    mc = torch.tensor(float(bank.mc[i]), dtype=torch.float64) * torch.exp(ln_mc - ln_mc.detach())
    m, kc, k, valid, Y = template_pixels(mc, torch.tensor(float(bank.eta[i]), dtype=torch.float64), f0,
                                         ct, ph, ps, torch.tensor(float(bank.cos_iota[i]), dtype=torch.float64),
                                         layout.m_end[li], grid, u, wm, weight_tf=weight_tf)
    z, N = _segment_sums(pix_t, m, k, valid, Y, layout.nseg[li], grid.n_tranches)
    ups = _upsilon(z, N)
    g = torch.ones_like(ups) if g_seg is None else torch.as_tensor(np.asarray(g_seg), dtype=torch.float64)
    L = (g * ups).sum()
    grads = torch.autograd.grad(L, [ln_mc, f0, ct, ph, ps])
    return np.array([float(x) for x in grads]), float(L.detach())


def forward_single(pix, u, wm, bank, grid, i: int, overrides=None):
    """Upsilon of template i with some parameters overridden (for finite differences).

    overrides: dict over PARAM_NAMES; ln_mc overrides set mc = exp(ln_mc).
    The integer structure is recomputed for the perturbed parameters.
    """
    b = bank.subset([i])
    if overrides:
        for key, val in overrides.items():
            if key == "ln_mc":
                b.mc = np.array([np.exp(val)])
            else:
                setattr(b, key, np.array([val]))
    res = statistic(pix, u, wm, b, grid)
    return res.stat[0], res
