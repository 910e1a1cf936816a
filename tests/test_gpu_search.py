"""Segment ladder on the GPU: candidates near the tiny injection refined from N_seg = 16 down to the coherent
N_seg = 1 (statistic, VJP and Adam step through the C ABI), with the final Upsilon_1 checked against the oracle."""
import numpy as np
import pytest

import tfsc_inputs as ti

from gpu_common import gridspec, lib, note, oracle_stat, rel, store_from_oracle, tiny_data

pytestmark = pytest.mark.gpu


def _starts(n, seed):
    """Starts about two resolution cells of the N_seg = 16 stage off the injection, sky angles 0.05 off."""
    inj = ti.TINY_INJECTION
    rng = np.random.default_rng(seed)
    return ti.Bank(mc=inj["mc"] * np.exp(rng.uniform(-2, 2, n) * 2.8e-3), eta=np.full(n, 0.25),
                   f0=inj["f0"] + rng.uniform(-2, 2, n) * 5e-7, cos_theta=np.full(n, inj["cos_theta"]) + 0.05,
                   phi=np.full(n, inj["phi"]) - 0.05, psi=np.full(n, inj["psi"]),
                   cos_iota=np.full(n, inj["cos_iota"]), phase=np.zeros(n))


def test_segment_ladder_climbs_to_the_coherent_peak():
    from paper_2510_19047_amd import search
    tfsc = lib()
    d = tiny_data()
    g = d["grid"]
    inj = ti.TINY_INJECTION
    n = 16
    b = _starts(n, 5)
    note("segment ladder 16 -> 8 -> 4 -> 2 -> 1 on the tiny injection")
    store = store_from_oracle(d, "f64")
    bt = tfsc.BankTensors.from_host(b)
    res = search.segment_ladder(gridspec(g), store, bt, ladder=(16, 8, 4, 2, 1), steps=30, lr_scale=0.5,
                                precision="f64")
    for ns, s0, s1 in zip(res.nseg, res.start, res.best):
        s0, s1 = s0.cpu().numpy(), s1.cpu().numpy()
        note(f"  N_seg {ns:3d}: start median {np.median(s0):8.1f}  best median {np.median(s1):8.1f}")
        assert np.all(s1 >= s0)
    # consecutive stages hand over the best point: a stage starts where the previous one's best was
    ups1 = res.upsilon1.cpu().numpy()
    np.testing.assert_array_equal(ups1, res.best[-1].cpu().numpy())
    # Upsilon_1 at the final parameters against the oracle (N_seg = 1)
    p = res.params.cpu().numpy()
    fin = ti.Bank(mc=p[:, 0], eta=b.eta, f0=p[:, 1], cos_theta=p[:, 2], phi=p[:, 3], psi=p[:, 4],
                  cos_iota=b.cos_iota, phase=b.phase)
    ref = oracle_stat(d, bank=fin, nseg_fixed=1)
    r = rel(ups1, ref.stat)
    note(f"  Upsilon_1 vs oracle: max rel {r.max():.2e}")
    assert r.max() < 1e-6
    # the coherent statistic at the injection's own parameters, and at the starting points
    exact = oracle_stat(d, bank=ti.tiny_bank().subset([256]), nseg_fixed=1).stat[0]
    start1 = oracle_stat(d, bank=b, nseg_fixed=1).stat
    df_start = np.abs(b.f0 - inj["f0"])
    df_end = np.abs(p[:, 1] - inj["f0"])
    note(f"  Upsilon_1: exact {exact:.1f}, start median {np.median(start1):.1f}, end median {np.median(ups1):.1f}; "
         f"|df0| median {np.median(df_start):.2e} -> {np.median(df_end):.2e}")
    assert np.median(ups1) > 0.9 * exact
    assert np.median(ups1 - start1) > 0.0
    assert np.median(df_end) < np.median(df_start)
    # the caller's bank is untouched
    assert np.array_equal(bt.f0.cpu().numpy(), b.f0)
