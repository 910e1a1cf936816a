"""Multi-harmonic templates: the statistic for a template made of several harmonics of the orbital phase.
Test infrastructure (the oracle), not part of the product path.

Paper passage followed: Sec. "Outlook" -- the time-frequency representation of the waveform extends to the
multi-harmonic case by computing the waveform quantities {A, f, fdot, phi} of every harmonic and applying the
Fresnel expressions (Eq. (fresnel-ft)) to each harmonic.  The sums of Eqs. (inner-tranche-tf),
(inner-segment-tf), (overlap-n) and (Upsilon-seg) are unchanged: they run over the template's pixels, which
are now the sum of the harmonics' pixels.

Readings fixed here (the paper prints no harmonic amplitudes or phasing beyond the Outlook's sentence):
* Harmonic h = 1, 2, ... of the orbital phase Phi / 2 has phase (h/2) Phi, frequency (h/2) f and chirp
  (h/2) fdot, with (Phi, f, fdot) the dominant (h = 2) harmonic's TaylorT3 track of ``oracle.track``; the
  factor h/2 is formed exactly (0.5 h) and multiplies each quantity once.
* Its strain is a_h A e^{i (h/2) Phi} with A = f^(2/3) the dominant harmonic's amplitude and a_h a complex
  factor given per template and harmonic (for eccentric binaries the caller's harmonic amplitudes); it carries
  the dominant harmonic's polarisation pattern (a+ = (1 + cos^2 iota)/2, ax = -i cos iota) and its own TDI
  transfer T_c(t_m, (h/2) f_m).  a_2 = 1 with every other a_h = 0 is the single-harmonic template.
* In tranche m harmonic h occupies its own N_F = 21 bins k_c,h - 10 .. k_c,h + 10, k_c,h = ceil(f_h dT),
  inside [1, M/2 - 1].  The template pixel of bin k is the sum over the harmonics whose window holds k; at
  low frequency the windows of neighbouring harmonics overlap and their values add there.
* The track ends before the first tranche where t_m + dT >= t_c, or where the highest harmonic h_max of the
  set violates the band or compactness condition: (h_max/2)(f_m + fdot_m dT) >= f_Nyq - 11 delta f or
  (h_max/2) fdot_m dT > 10 delta f.  N_seg is the dominant harmonic's (``oracle.track.nseg_rule``).

The template column of a tranche is built densely over all bins (each harmonic's 21 values added at their
bins), so the statistic needs no bookkeeping of overlaps: z_n = sum conj(D) Y and N_n = sum |Y|^2 over the
dense columns of the segment's tranches, Upsilon_n = 2 |z_n|^2 / N_n.
"""
from __future__ import annotations

import numpy as np
import torch

from . import track as trk
from .fresnel import tranche_spectrum
from .response import transfer_aet

NF_HALF = 10


def check_harmonics(harmonics) -> np.ndarray:
    h = np.asarray(harmonics, dtype=np.int64)
    if h.ndim != 1 or h.size < 1 or np.any(h < 1) or np.any(h > 8) or np.unique(h).size != h.size:
        raise ValueError("harmonics: 1 to 8 distinct harmonic numbers of the orbital phase, each in 1..8")
    return h


def track_end(bank, grid, harmonics, layout: trk.Layout | None = None):
    """(m_end, flags) per template: the single-harmonic layout's merger condition, with the band and
    compactness conditions applied to the highest harmonic of the set."""
    h = check_harmonics(harmonics)
    lay = trk.Layout(bank, grid) if layout is None else layout
    smax = 0.5 * float(h.max())
    dT = float(grid.tranche_dur)
    df = 1.0 / dT
    fnyq = 0.5 / grid.dt
    Nt = grid.n_tranches
    tm = torch.arange(Nt, dtype=torch.float64) * dT
    m_end = np.zeros(lay.n, dtype=np.int64)
    flags = np.zeros(lay.n, dtype=np.int64)
    for i in range(lay.n):
        if not lay.valid[i]:
            flags[i] = trk.FLAG_INVALID
            continue
        tpl = lay.template(i)
        tc = float(tpl.tc)
        merge = (tm + dT) >= tc
        safe_t = torch.where(merge, torch.zeros_like(tm), tm)
        _, f, fdot, _ = tpl.at(safe_t)
        band = (smax * (f + fdot * dT)) >= (fnyq - 11.0 * df)
        compact = (smax * fdot * dT) > (10.0 * df)
        stop = torch.nonzero(merge | band | compact)
        if stop.numel() == 0:
            m_end[i] = Nt
        else:
            m = int(stop[0])
            m_end[i] = m
            flags[i] |= trk.FLAG_MERGE_END if bool(merge[m]) else trk.FLAG_BAND_END
        if m_end[i] == 0:
            flags[i] |= trk.FLAG_EMPTY
    return m_end, flags, lay


def harmonic_pixels(mc, eta, f0, cos_theta, phi, psi, cos_iota, m_end: int, grid, u, wm, harmonics, amps,
                    exact_fresnel: bool = False):
    """Per-harmonic template pixels of one template: a list over the harmonics of (k[n_m, 21], valid[n_m, 21],
    Y[C, n_m, 21]) on the active tranches m = 0 .. m_end - 1, with Y = a_h T_c(t_m, f_h) h_h(f_k) u_k w_m."""
    dT = float(grid.tranche_dur)
    M = grid.tranche_len
    m = torch.arange(int(m_end), dtype=torch.int64)
    tm = m.to(torch.float64) * dT
    Phi, f, fdot, A = trk.Template(mc, eta, f0).at(tm)
    w = torch.as_tensor(np.asarray(wm), dtype=torch.float64)[m]
    uk_all = torch.as_tensor(np.asarray(u), dtype=torch.float64)
    out = []
    for hh, a in zip(check_harmonics(harmonics), np.asarray(amps, dtype=np.complex128)):
        s = 0.5 * float(hh)
        Ph, fh, fdh = s * Phi, s * f, s * fdot
        with torch.no_grad():
            kc = torch.ceil(fh * dT).to(torch.int64)
        k = kc[:, None] + torch.arange(-NF_HALF, NF_HALF + 1, dtype=torch.int64)[None, :]
        valid = (k >= 1) & (k <= M // 2 - 1)
        fk = k.to(torch.float64) / dT
        spec = tranche_spectrum(Ph[:, None], fh[:, None], fdh[:, None], A[:, None], fk, dT, exact=exact_fresnel)
        T = list(transfer_aet(tm, fh, cos_theta, phi, psi, cos_iota))[: grid.n_channels]
        weight = torch.where(valid, uk_all[k.clamp(0, M // 2)], torch.zeros(k.shape, dtype=torch.float64))
        weight = weight * w[:, None]
        aa = complex(a)
        Y = torch.stack([aa * Tc[:, None] * spec * weight for Tc in T], dim=0)
        out.append((k, valid, Y))
    return m, out


def dense_columns(m, per_harmonic, n_bins: int, n_channels: int):
    """The template column of every active tranche over all bins: Y[C, n_m, K], the harmonics' windows added."""
    cols = torch.zeros((n_channels, m.numel(), n_bins), dtype=torch.complex128)
    rows = torch.arange(m.numel(), dtype=torch.int64)[:, None]
    for k, valid, Y in per_harmonic:
        kk = torch.where(valid, k, torch.zeros_like(k))
        for c in range(n_channels):
            add = torch.where(valid, Y[c], torch.zeros_like(Y[c]))
            cols[c].index_put_((rows.expand_as(kk), kk), add, accumulate=True)
    return cols


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


def statistic(pix, u, wm, bank, grid, harmonics, amps, exact_fresnel: bool = False, idx=None) -> Result:
    """Upsilon and its per-segment terms of every template of ``bank`` made of the given harmonics.

    pix: whitened data pixels [C][K][Nt]; u [K], wm [Nt] as in ``oracle.o2``; harmonics: [H] harmonic numbers
    of the orbital phase; amps: complex [n][H] factors a_h per template (or [H], the same for every template).
    """
    h = check_harmonics(harmonics)
    amps = np.asarray(amps, dtype=np.complex128)
    if amps.ndim == 1:
        amps = np.broadcast_to(amps, (len(bank.mc), h.size))
    m_end, flags, lay = track_end(bank, grid, h)
    res = Result(lay.n, lay.seg_offset)
    res.m_end[:] = m_end
    res.nseg[:] = lay.nseg
    res.flags[:] = flags
    pix_t = torch.as_tensor(np.asarray(pix, dtype=np.complex128))
    C, K, Nt = pix_t.shape
    rows = range(lay.n) if idx is None else idx
    with torch.no_grad():
        for i in rows:
            if flags[i] & (trk.FLAG_INVALID | trk.FLAG_EMPTY):
                continue
            m, per = harmonic_pixels(bank.mc[i], bank.eta[i], bank.f0[i], bank.cos_theta[i], bank.phi[i],
                                     bank.psi[i], bank.cos_iota[i], m_end[i], grid, u, wm, h, amps[i],
                                     exact_fresnel)
            Y = dense_columns(m, per, K, C)                      # [C, n_m, K]
            D = pix_t[:, :, : m.numel()].permute(0, 2, 1)        # [C, n_m, K]
            keep = torch.zeros(K, dtype=torch.bool)
            keep[1: grid.tranche_len // 2] = True                # DC and Nyquist never enter
            D = torch.where(keep[None, None, :], D, torch.zeros_like(D))
            zm = (torch.conj(D) * Y).sum(dim=(0, 2))
            Nm = (Y.real * Y.real + Y.imag * Y.imag).sum(dim=(0, 2))
            ns = int(lay.nseg[i])
            seg = (m * ns) // int(Nt)
            z = torch.zeros(ns, dtype=torch.complex128).index_add(0, seg, zm)
            N = torch.zeros(ns, dtype=torch.float64).index_add(0, seg, Nm)
            zz = z.real * z.real + z.imag * z.imag
            ups = torch.where(N > 0, 2.0 * zz / torch.where(N > 0, N, torch.ones_like(N)), torch.zeros_like(N))
            o = lay.seg_offset[i]
            res.seg_terms[o:o + ns] = ups.numpy()
            res.seg_z[o:o + ns] = z.numpy()
            res.seg_N[o:o + ns] = N.numpy()
            res.stat[i] = float(ups.sum())
            if not bool((N > 0).any()):
                res.flags[i] |= trk.FLAG_ALL_EXCLUDED
    return res


def template_column_pixels(bank, i: int, grid, u, wm, harmonics, amps):
    """Dense template pixels [C][K][Nt] of template i (zero outside its active tranches): for pixel-domain
    injections of a multi-harmonic signal."""
    h = check_harmonics(harmonics)
    sub = bank.subset([i])
    m_end, flags, _ = track_end(sub, grid, h)
    C, K, Nt = grid.n_channels, grid.tranche_len // 2 + 1, grid.n_tranches
    out = np.zeros((C, K, Nt), dtype=np.complex128)
    if flags[0] & (trk.FLAG_INVALID | trk.FLAG_EMPTY):
        return out
    with torch.no_grad():
        m, per = harmonic_pixels(sub.mc[0], sub.eta[0], sub.f0[0], sub.cos_theta[0], sub.phi[0], sub.psi[0],
                                 sub.cos_iota[0], m_end[0], grid, u, wm, h, np.asarray(amps, np.complex128))
        Y = dense_columns(m, per, K, C).numpy()
    out[:, :, : Y.shape[1]] = np.transpose(Y, (0, 2, 1))
    return out
