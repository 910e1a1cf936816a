"""The plain-C O2 agrees with the torch O2: integers bit for bit, the statistic to 1e-12 (CPU)."""
import ctypes

import numpy as np
import torch

import tfsc_inputs as ti
from oracle import cpu, o2
from oracle import track as trk
from oracle import transform as tf


def _check(rc, r2, n):
    assert np.array_equal(rc.m_end, r2.m_end)
    assert np.array_equal(rc.nseg, r2.nseg)
    assert np.array_equal(rc.flags, r2.flags)
    assert np.max(np.abs(rc.stat - r2.stat) / np.maximum(np.abs(r2.stat), 1.0)) < 1e-12
    assert np.max(np.abs(rc.seg_terms - r2.seg_terms)) < 1e-12 * max(1.0, np.max(r2.seg_terms))


def test_tiny_bank(tiny_setup):
    s = tiny_setup
    r2 = o2.statistic(s["pix"], s["u"], s["wm"], s["bank"], s["grid"])
    rc = cpu.statistic(s["pix"], s["u"], s["wm"], s["bank"], s["grid"], threads=4)
    _check(rc, r2, len(s["bank"]))


def test_two_channel_gapped_with_invalid_rows(small_grid):
    g = small_grid
    b = ti.random_bank(40, 9, mc_range=(5.0, 100.0), f0_range=(0.003, 0.09), stream=51)
    b.mc[3] = 0.0
    b.eta[4] = 0.26
    b.f0[5] = 0.3
    b.cos_theta[6] = 1.2
    psd = ti.psd_on_bins(g)
    mu, keep = ti.tranche_psd_scale(g), ti.tranche_keep(g)
    _, u, wm = tf.whitening(g.tranche_len, g.dt, 0.1, psd, mu, keep)
    pix = ti.pixel_noise((2, g.n_bins, g.n_tranches), stream=52)
    r2 = o2.statistic(pix, u, wm, b, g)
    rc = cpu.statistic(pix, u, wm, b, g, threads=4, want_zn=True)
    _check(rc, r2, len(b))
    assert np.allclose(rc.seg_zn[:, 0] + 1j * rc.seg_zn[:, 1], r2.seg_z, rtol=1e-11, atol=1e-12)
    assert np.allclose(rc.seg_zn[:, 2], r2.seg_N, rtol=1e-11, atol=0)
    assert rc.flags[3] == trk.FLAG_INVALID and rc.flags[4] == trk.FLAG_INVALID and rc.flags[6] == trk.FLAG_INVALID
    assert rc.flags[5] & trk.FLAG_EMPTY
    assert (rc.flags & trk.FLAG_BAND_END).any()


def test_c_track_bit_exact_with_torch_track():
    L = cpu.lib()
    P = ctypes.c_void_p
    L.o2_cpu_track.argtypes = [ctypes.c_double] * 3 + [ctypes.c_int64, P, P, P]
    b = ti.random_bank(20, 9, mc_range=(5.0, 100.0), f0_range=(0.002, 0.05), stream=53)
    for i in range(len(b)):
        T = trk.Template(torch.tensor(b.mc[i], dtype=torch.float64), torch.tensor(b.eta[i], dtype=torch.float64),
                         torch.tensor(b.f0[i], dtype=torch.float64))
        t = np.linspace(0.0, 0.95 * float(T.tc), 301)
        out = np.zeros((t.size, 4))
        tc = np.zeros(1)
        L.o2_cpu_track(b.mc[i], b.eta[i], b.f0[i], t.size, t.ctypes.data_as(P), out.ctypes.data_as(P),
                       tc.ctypes.data_as(P))
        Phi, f, fdot, A = T.at(torch.tensor(t))
        assert tc[0] == float(T.tc)
        assert np.array_equal(out[:, 0], Phi.numpy())
        assert np.array_equal(out[:, 1], f.numpy())
        assert np.array_equal(out[:, 2], fdot.numpy())
