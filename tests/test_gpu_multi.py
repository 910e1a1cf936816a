"""Several noise realisations in one pass over the bank (tfsc_bank_statistic_multi through the C ABI) against
the single-realisation statistic and the oracle."""
import numpy as np
import pytest
import torch

import tfsc_inputs as ti

from gpu_common import dev, gridspec, lib, note, oracle_stat, rel, small_data

pytestmark = pytest.mark.gpu


def _stores(tfsc, g, d, R, dtype, layout):
    keep = ti.sample_keep_mask(g)[None, :]
    stores = tfsc.realisation_stores(gridspec(g), R, dtype=dtype, layout=layout)
    xs = []
    for r in range(R):
        x = ti.noise(g, realisation=r) * keep
        x = x.astype(np.float64 if dtype == "f64" else np.float32)
        xs.append(x)
        tfsc.transform(gridspec(g), dev(x), dev(d["psd"]), dev(d["mu"]), dev(d["keep"]), dtype=dtype, out=stores[r])
    return stores, xs


@pytest.mark.parametrize("layout,group", [("layer_ci", 0), ("layer_ci", 8), ("layer", 4)])
def test_multi_matches_single_realisation_fp32(layout, group):
    """11 realisations in groups (2: five pairs and one alone; 8: eight, then 2 and 1; 4: 4, 4, 2, 1) against
    eleven single launches."""
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    R = 11
    note(f"multi-realisation statistic, {R} realisations, f32 {layout}, group {group}")
    stores, _ = _stores(tfsc, g, d, R, "f32", layout)
    bt = tfsc.BankTensors.from_host(d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt)
    order = tfsc.processing_order(gridspec(g), bt)
    res = tfsc.bank_statistic_multi(gridspec(g), stores, bt, seg, precision="f32", order=order, want_active=True,
                                    group=group)
    worst = 0.0
    for r in range(R):
        one = tfsc.bank_statistic(gridspec(g), stores[r], bt, seg, precision="f32", schedule="wave",
                                  want_active=True)
        a, b = res.stat[r].cpu().numpy(), one.stat.cpu().numpy()
        worst = max(worst, rel(a, b).max())
        assert rel(a, b).max() < 2e-6, r
        st_a, st_b = res.seg_terms[r, :seg.total].cpu().numpy(), one.seg_terms[:seg.total].cpu().numpy()
        assert np.max(np.abs(st_a - st_b) / np.maximum(st_b, 1.0)) < 2e-5, r
        if r == 0:
            assert torch.equal(res.flags, one.flags) and torch.equal(res.n_active, one.n_active)
    note(f"  max rel against single launches {worst:.2e}")
    # realisations differ
    assert not torch.equal(res.stat[0], res.stat[1])


def test_multi_fp64_against_oracle_and_low_frequency_rows():
    """FP64 pixels and arithmetic, 9 realisations (a group of eight and one alone), on a bank whose tracks start
    near bin 2 (the per-lane row path) plus the small bank: realisations 0 and 8 against the oracle at 1e-6."""
    from oracle import transform as otf
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    R = 9
    note("multi-realisation statistic, f64, low-frequency and wide banks")
    stores, xs = _stores(tfsc, g, d, R, "f64", "layer_ci")
    low = ti.random_bank(128, 7, mc_range=(5.0, 100.0), f0_range=(0.0008, 0.006), eta=None, stream=33)
    bank = ti.Bank.concat(low, d["bank"])
    bt = tfsc.BankTensors.from_host(bank)
    seg = tfsc.segment_layout(gridspec(g), bt)
    res = tfsc.bank_statistic_multi(gridspec(g), stores, bt, seg, precision="f64", group=8)
    for r in (0, R - 1):
        pix, u, wm = otf.transform(xs[r], g, d["psd"], d["mu"], d["keep"], 0.1, "rfft")
        ref = oracle_stat(dict(d, pix=pix, u=u, wm=wm), bank=bank)
        s = res.stat[r].cpu().numpy()
        # the float64 oracle's own small-beta loss reaches ~2e-6 on the lowest templates
        r_all = rel(s, ref.stat)
        note(f"  realisation {r}: max rel vs oracle {r_all.max():.2e} (wide bank {r_all[128:].max():.2e})")
        assert r_all[128:].max() < 1e-6
        assert r_all.max() < 3e-6
        assert np.array_equal(res.flags.cpu().numpy(), ref.flags)


def test_multi_argument_errors():
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    bt = tfsc.BankTensors.from_host(d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt)
    stores, _ = _stores(tfsc, g, d, 2, "f32", "layer_ci")
    with pytest.raises(tfsc.TfscError):  # FP32 pixels with FP64 arithmetic
        tfsc.bank_statistic_multi(gridspec(g), stores, bt, seg, precision="f64")
    t = tfsc.transform(gridspec(g), dev(d["x"].astype(np.float32)), dev(d["psd"]), dev(d["mu"]), dev(d["keep"]),
                       dtype="f32", layout="tranche")
    with pytest.raises(tfsc.TfscError):  # tranche-major store
        tfsc.bank_statistic_multi(gridspec(g), [t], bt, seg)
    with pytest.raises(tfsc.TfscError):  # stores not at one stride
        tfsc.bank_statistic_multi(gridspec(g), [stores[0], stores[1], stores[0]], bt, seg)
    with pytest.raises(tfsc.TfscError):  # group size
        tfsc.bank_statistic_multi(gridspec(g), stores, bt, seg, group=3)


@pytest.mark.parametrize("dtype", ["f32", "i16"])
@pytest.mark.parametrize("channels,n_real", [(2, 2), (2, 4), (1, 2), (1, 4)])
def test_interleaved_realisations_match_single_launches(channels, n_real, dtype):
    """Realisations interleaved cell by cell in one FP32 or int16 store (real_stride 0): each realisation against
    its own single-realisation launch on the same pixels (2e-6; the same bin sums, FMA contraction may differ),
    on the small bank plus a bank whose tracks start near bin 2 (the per-lane row path); flags and active
    counts equal; realisation 0 against the oracle (FP32: 1e-6 on the wide bank, the float64 oracle's own
    small-beta loss on the low one; int16: the store's 1e-4 bar)."""
    from oracle import transform as otf
    tfsc = lib()
    d = small_data()
    g0 = d["grid"]
    g = g0 if channels == 2 else ti.custom_grid(1, g0.tranche_len, g0.n_tranches, dt=g0.dt, modulated=True,
                                                   gapped=True, cfg_id=g0.cfg_id)
    note(f"interleaved realisations: C={channels}, {n_real} realisations, {dtype}")
    keep = ti.sample_keep_mask(g)[None, :]
    xs = [(ti.noise(g, realisation=r) * keep).astype(np.float32) for r in range(n_real)]
    psd, mu, kp = ti.psd_on_bins(g), ti.tranche_psd_scale(g), ti.tranche_keep(g)
    stores = [tfsc.transform(gridspec(g), dev(x), dev(psd), dev(mu), dev(kp), dtype=dtype, layout="layer_ci")
              for x in xs]
    ri = tfsc.interleave_stores(gridspec(g), stores)
    low = ti.random_bank(64, 7, mc_range=(5.0, 100.0), f0_range=(0.0008, 0.006), eta=None, stream=35)
    bank = ti.Bank.concat(low, d["bank"])
    bt = tfsc.BankTensors.from_host(bank)
    seg = tfsc.segment_layout(gridspec(g), bt)
    order = tfsc.processing_order(gridspec(g), bt)
    res = tfsc.bank_statistic_interleaved(gridspec(g), ri, n_real, bt, seg, order=order, want_active=True)
    worst = 0.0
    for r in range(n_real):
        one = tfsc.bank_statistic(gridspec(g), stores[r], bt, seg, precision="f32", schedule="wave", want_active=True)
        a, b = res.stat[r].cpu().numpy(), one.stat.cpu().numpy()
        worst = max(worst, rel(a, b).max())
        assert rel(a, b).max() < 2e-6, r
        st_a, st_b = res.seg_terms[r, :seg.total].cpu().numpy(), one.seg_terms[:seg.total].cpu().numpy()
        assert np.max(np.abs(st_a - st_b) / np.maximum(st_b, 1.0)) < 2e-5, r
        assert torch.equal(res.flags, one.flags) and torch.equal(res.n_active, one.n_active)
    pix, u, wm = otf.transform(xs[0].astype(np.float64), g, psd, mu, kp, 0.1, "rfft")
    ref = oracle_stat(dict(d, grid=g, pix=pix, u=u, wm=wm), bank=bank)
    r0 = rel(res.stat[0].cpu().numpy(), ref.stat)
    note(f"  max rel against single launches {worst:.2e}; realisation 0 vs oracle {r0.max():.2e} "
         f"(wide bank {r0[64:].max():.2e})")
    if dtype == "f32":
        assert r0[64:].max() < 1e-6 and r0.max() < 3e-6
    else:
        assert r0.max() < 1e-4
    assert np.array_equal(res.flags.cpu().numpy(), ref.flags)
    assert not torch.equal(res.stat[0], res.stat[1])


def test_interleaved_argument_errors():
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    bt = tfsc.BankTensors.from_host(d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt)
    x = dev(d["x"].astype(np.float32))
    s = tfsc.transform(gridspec(g), x, dev(d["psd"]), dev(d["mu"]), dev(d["keep"]), dtype="f32", layout="layer_ci")
    ri = tfsc.interleave_stores(gridspec(g), [s, s, s])
    with pytest.raises(tfsc.TfscError):  # three realisations interleaved
        tfsc.bank_statistic_interleaved(gridspec(g), ri, 3, bt, seg)
    lay = tfsc.transform(gridspec(g), x, dev(d["psd"]), dev(d["mu"]), dev(d["keep"]), dtype="f32", layout="layer")
    with pytest.raises(tfsc.TfscError):  # only channel-interleaved stores interleave
        tfsc.interleave_stores(gridspec(g), [lay, lay])
    h = tfsc.transform(gridspec(g), x, dev(d["psd"]), dev(d["mu"]), dev(d["keep"]), dtype="f16", layout="layer_ci")
    with pytest.raises(tfsc.TfscError):  # FP32 and int16 stores only
        tfsc.interleave_stores(gridspec(g), [h, h])
