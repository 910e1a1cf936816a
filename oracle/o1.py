"""O1: the statistic from its definition.

Paper passages followed: Eqs. (inner), (inner-segment), (overlap-n),
(Upsilon-seg) define the statistic through discrete Fourier transforms of
the data and of the template's TDI response; Sec. "Implementation details"
defines the data model (TDI A/E of the dominant-mode strain through the
single-link responses of the constellation).  O1 evaluates those
definitions directly:

1. the template's strain (TaylorT3 phase, amplitude f^(2/3), polarisation
   amplitudes (1 + cos^2 iota)/2 and cos iota) is evaluated at every
   delayed time each single link needs, and TDI A/E are formed sample by
   sample (``oracle.response.tdi_aet_td``) -- no Taylor expansion, no
   Fresnel forms, no per-tranche transfer function;
2. every tranche of the template and of the data is transformed by the
   direct DFT of ``oracle.transform``; template pixels are weighted by
   u_k w_m like the data's whitening;
3. per segment z_n = sum conj(D) Y and N_n = sum |Y|^2 over channels,
   tranches and a bin set K_m (all bins 1..M/2-1, or the 21 bins of the
   track), and Upsilon = sum_n 2 |z_n|^2 / N_n.

The signal is switched off at the end of the template's last active
tranche (the track-end rule of ``oracle.track``).  ``analytic=True``
synthesises the complex positive-frequency strain A e^{i Phi} (for
pixel-level comparisons with O2); ``analytic=False`` the real strain.
"""
from __future__ import annotations

import numpy as np
import torch

from . import track as trk
from .response import tdi_aet_td
from .transform import tranche_dft


def strain_callback(tpl: trk.Template, cos_iota: float, t_stop: float, phase: float = 0.0,
                    analytic: bool = False, amp: float = 1.0, harmonics=None):
    """(h+, hx) at delayed times.  ``harmonics`` = (h[H], a[H]): the strain sum_h a_h A e^{i (h/2) Phi} over
    harmonics of the orbital phase (Sec. "Outlook"), each with the dominant harmonic's polarisation pattern;
    None is the dominant harmonic alone (h = 2, a = 1)."""
    ci = float(cos_iota)
    ap = (1.0 + ci * ci) / 2.0
    hs = [(1.0, 1.0 + 0.0j)] if harmonics is None else [(0.5 * float(h), complex(a)) for h, a in zip(*harmonics)]

    def hfun(tq):
        on = tq < t_stop
        tsafe = torch.where(on, tq, torch.zeros_like(tq))
        Phi, f, fdot, A = tpl.at(tsafe)
        A = torch.where(on, A * amp, torch.zeros_like(A))
        if harmonics is None:
            Phi = Phi + phase
            if analytic:
                e = torch.polar(torch.ones_like(Phi), Phi)
                return A * ap * e, A * torch.complex(torch.zeros_like(Phi), -ci * torch.ones_like(Phi)) * e
            return A * ap * torch.cos(Phi), A * ci * torch.sin(Phi)
        w = torch.zeros(Phi.shape, dtype=torch.complex128)
        for s, a in hs:
            ph = s * Phi + phase
            w = w + a * torch.polar(torch.ones_like(ph), ph)
        hp = A * ap * w
        hx = A * torch.complex(torch.zeros_like(Phi), -ci * torch.ones_like(Phi)) * w
        if analytic:
            return hp, hx
        return hp.real, hx.real

    return hfun


def synthesize(bank, i: int, grid, analytic: bool = False, t_stop: float | None = None,
               amp: float = 1.0, chunk: int = 1 << 18, harmonics=None) -> np.ndarray:
    """TDI [C][N] time series of source i of ``bank`` (phase offset from bank.phase if set).  ``harmonics`` =
    (h[H], a[H]) synthesises a multi-harmonic source; it then stops where the highest harmonic's track ends."""
    lay = trk.Layout(bank.subset([i]), grid)
    tpl = lay.template(0)
    if t_stop is None:
        if harmonics is None:
            t_stop = float(lay.m_end[0]) * grid.tranche_dur
        else:
            from .harmonics import track_end
            m_end, _, _ = track_end(bank.subset([i]), grid, harmonics[0], layout=lay)
            t_stop = float(m_end[0]) * grid.tranche_dur
    phase = 0.0 if bank.phase is None else float(bank.phase[i])
    hfun = strain_callback(tpl, bank.cos_iota[i], t_stop, phase, analytic, amp, harmonics)
    N = grid.n_samples
    dtype = np.complex128 if analytic else np.float64
    out = np.zeros((grid.n_channels, N), dtype=dtype)
    for s in range(0, N, chunk):
        e = min(N, s + chunk)
        t = torch.arange(s, e, dtype=torch.float64) * grid.dt
        A, E, T = tdi_aet_td(t, hfun, bank.cos_theta[i], bank.phi[i], bank.psi[i])
        out[0, s:e] = A.numpy()
        if grid.n_channels > 1:
            out[1, s:e] = E.numpy()
        if grid.n_channels > 2:
            out[2, s:e] = T.numpy()
    return out


def template_pixels(bank, i: int, grid, u, wm, alpha: float = 0.0, harmonics=None) -> np.ndarray:
    """Y[C][K][Nt] = DFT of the analytic TD template (window alpha) times u_k w_m, times dt.

    The factor dt makes the DFT approximate the continuous transform, which is
    the normalisation of the Fresnel-kernel spectrum of O2.
    """
    x = synthesize(bank, i, grid, analytic=True, harmonics=harmonics)
    M = grid.tranche_len
    Y = np.empty((grid.n_channels, M // 2 + 1, grid.n_tranches), dtype=np.complex128)
    for c in range(grid.n_channels):
        Y[c] = tranche_dft(x[c], M, alpha, "direct") * grid.dt
    return Y * np.asarray(u)[None, :, None] * np.asarray(wm)[None, None, :]


def bin_mask(grid, lay: trk.Layout, li: int, which: str = "21") -> np.ndarray:
    """Boolean [K][Nt]: bins used per tranche (active tranches only)."""
    M = grid.tranche_len
    K = M // 2 + 1
    mask = np.zeros((K, grid.n_tranches), dtype=bool)
    m_end = int(lay.m_end[li])
    if m_end == 0:
        return mask
    if which == "full":
        mask[1:M // 2, :m_end] = True
        return mask
    tpl = lay.template(li)
    tm = torch.arange(m_end, dtype=torch.float64) * grid.tranche_dur
    _, f, _, _ = tpl.at(tm)
    kc = torch.ceil(f * grid.tranche_dur).to(torch.int64).numpy()
    for j in range(-10, 11):
        k = kc + j
        ok = (k >= 1) & (k <= M // 2 - 1)
        mask[k[ok], np.arange(m_end)[ok]] = True
    return mask


def statistic_from_pixels(D: np.ndarray, Y: np.ndarray, mask: np.ndarray, nseg: int, Nt: int):
    """Per-segment (z_n, N_n, Upsilon_n) from full-grid pixels restricted to mask."""
    seg = (np.arange(Nt) * int(nseg)) // int(Nt)
    z = np.zeros(int(nseg), dtype=np.complex128)
    N = np.zeros(int(nseg))
    prod = (np.conj(D) * Y).sum(axis=0)
    pw = (np.abs(Y) ** 2).sum(axis=0)
    zm = np.where(mask, prod, 0).sum(axis=0)
    Nm = np.where(mask, pw, 0).sum(axis=0)
    np.add.at(z, seg, zm)
    np.add.at(N, seg, Nm)
    ups = np.where(N > 0, 2.0 * np.abs(z) ** 2 / np.where(N > 0, N, 1.0), 0.0)
    return z, N, ups
