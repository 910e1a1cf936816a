"""Shared set-up for the GPU parity tests: seeded inputs, oracle results, device copies."""
from __future__ import annotations

import functools
import sys

import numpy as np
import torch

import tfsc_inputs as ti
from oracle import cpu as ocpu
from oracle import o2
from oracle import track as otrk
from oracle import transform as otf


def note(msg: str):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def lib():
    import paper_2510_19047_amd as tfsc
    tfsc.lib()  # raises if the HIP library is missing
    return tfsc


def gridspec(g, alpha=0.1):
    tfsc = lib()
    return tfsc.GridSpec(g.n_channels, g.tranche_len, g.n_tranches, g.dt, alpha)


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


@functools.lru_cache(maxsize=4)
def tiny_data(alpha: float = 0.1):
    """Tiny workload: noise + the SNR-20 injection (time domain, oracle O1), oracle pixels."""
    from oracle import o1
    g = ti.TINY
    psd = ti.psd_on_bins(g)
    mu, keep = ti.tranche_psd_scale(g), ti.tranche_keep(g)
    inj = ti.tiny_injection()
    sig = o1.synthesize(inj, 0, g, analytic=False)
    spix, _, _ = otf.transform(sig, g, psd, mu, keep, alpha, "rfft")
    rho = np.sqrt(2 * np.sum(np.abs(spix[:, 1:-1]) ** 2))
    x = ti.noise(g) + sig * (ti.TINY_INJECTION["snr"] / rho)
    pix, u, wm = otf.transform(x, g, psd, mu, keep, alpha, "rfft")
    return dict(grid=g, x=x, psd=psd, mu=mu, keep=keep, pix=pix, u=u, wm=wm, bank=ti.tiny_bank(), alpha=alpha)


@functools.lru_cache(maxsize=4)
def small_data(n_templates: int = 96, seed_stream: int = 61):
    """Two channels, gaps and PSD modulation; a wide random bank with invalid and empty rows."""
    g = ti.custom_grid(2, 512, 700, dt=5.0, modulated=True, gapped=True, cfg_id=7)
    psd = ti.psd_on_bins(g)
    mu, keep = ti.tranche_psd_scale(g), ti.tranche_keep(g)
    x = ti.noise(g)
    pix, u, wm = otf.transform(x, g, psd, mu, keep, 0.1, "rfft")
    b = ti.random_bank(n_templates, 7, mc_range=(5.0, 100.0), f0_range=(0.004, 0.08), eta=None, stream=seed_stream)
    b.mc[3] = -2.0            # invalid
    b.eta[5] = 0.3            # invalid
    b.f0[7] = 0.2             # above Nyquist: empty track
    b.cos_iota[9] = 1.0       # face-on
    return dict(grid=g, x=x, psd=psd, mu=mu, keep=keep, pix=pix, u=u, wm=wm, bank=b)


def oracle_stat(d, bank=None, nseg_fixed=None, want_zn=False):
    b = d["bank"] if bank is None else bank
    return ocpu.statistic(d["pix"], d["u"], d["wm"], b, d["grid"], nseg_fixed=nseg_fixed, threads=0, want_zn=want_zn)


def store_from_oracle(d, dtype="f64", layout="layer"):
    tfsc = lib()
    return tfsc.PixelStore.from_complex(dev(d["pix"]), dev(d["u"]), dev(d["wm"]), dtype=dtype, layout=layout)


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), 1.0)


@functools.lru_cache(maxsize=1)
def full_injected():
    """The full-size data (2-yr A+E, gaps, modulated PSD; noise stream 0) with the 20 injections of the full-size
    configuration added in the pixel domain (the oracle's own template pixels, phase-shifted and scaled to their
    target SNR): oracle pixels, weights and the injection parameters."""
    g = ti.FULL
    note("full-size data: noise + 20 pixel-domain injections")
    x = ti.noise(g) * ti.sample_keep_mask(g)[None, :]
    psd, mu, keep = ti.psd_on_bins(g), ti.tranche_psd_scale(g), ti.tranche_keep(g)
    pix, u, wm = otf.transform(x, g, psd, mu, keep, 0.1, "rfft")
    inj, snr = ti.full_injections()
    lay = otrk.Layout(inj, g)
    K = g.tranche_len // 2 + 1
    with torch.no_grad():
        for i in range(len(inj)):
            if lay.flags[i] & (otrk.FLAG_INVALID | otrk.FLAG_EMPTY):
                continue
            m, kc, k, valid, Y = o2.template_pixels(inj.mc[i], inj.eta[i], inj.f0[i], inj.cos_theta[i], inj.phi[i],
                                                    inj.psi[i], inj.cos_iota[i], lay.m_end[i], g, u, wm)
            Y = Y.numpy() * np.exp(1j * inj.phase[i])
            rho = np.sqrt(2.0 * np.sum(np.abs(Y) ** 2))
            Y *= snr[i] / rho
            kk = np.clip(k.numpy(), 0, K - 1)
            mm = np.broadcast_to(m.numpy()[:, None], kk.shape)
            v = valid.numpy()
            for c in range(g.n_channels):
                np.add.at(pix[c], (kk[v], mm[v]), Y[c][v])
    return dict(grid=g, pix=pix, u=u, wm=wm, inj=inj, snr=snr)
