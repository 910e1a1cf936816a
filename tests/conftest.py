import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU; runs the HIP path")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def tiny_setup():
    """Tiny workload: noise-only whitened pixels of channel A plus the bank (oracle transform)."""
    import tfsc_inputs as ti
    from oracle import transform as tf
    g = ti.TINY
    psd = ti.psd_on_bins(g)
    mu = ti.tranche_psd_scale(g)
    keep = ti.tranche_keep(g)
    x = ti.noise(g)
    pix, u, wm = tf.transform(x, g, psd, mu, keep, 0.1, "rfft")
    return dict(grid=g, psd=psd, mu=mu, keep=keep, x=x, pix=pix, u=u, wm=wm, bank=ti.tiny_bank())


@pytest.fixture(scope="session")
def small_grid():
    """A small 2-channel grid with gaps and modulation for fast pixel-domain checks."""
    import tfsc_inputs as ti
    return ti.custom_grid(2, 512, 160, dt=5.0, modulated=True, gapped=True)


def rel_err(a, b, floor=1.0):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), floor)
