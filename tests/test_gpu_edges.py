"""Edge cases of the statistic through the C ABI: every tranche excluded, one tranche per segment, and a single
channel in the channel-interleaved layout."""
import numpy as np
import pytest
import torch

from oracle import track as otrk

from gpu_common import dev, gridspec, lib, note, oracle_stat, rel, small_data, store_from_oracle, tiny_data

pytestmark = pytest.mark.gpu


def test_every_tranche_excluded():
    """All tranche weights 0 (as if the whole span were gapped): every valid template that reaches a tranche is
    flagged ALL_EXCLUDED with Upsilon = 0, on both schedules and in the several-realisation form, as in the
    oracle."""
    tfsc = lib()
    d = dict(small_data())
    d["wm"] = np.zeros_like(d["wm"])
    g = d["grid"]
    note("all tranches excluded")
    ref = oracle_stat(d)
    assert np.any(ref.flags & otrk.FLAG_ALL_EXCLUDED)
    bt = tfsc.BankTensors.from_host(d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt)
    for schedule, layout in (("thread", "tranche"), ("wave", "layer_ci")):
        res = tfsc.bank_statistic(gridspec(g), store_from_oracle(d, "f32", layout=layout), bt, seg, precision="f32",
                                  schedule=schedule, want_active=True)
        assert np.array_equal(res.flags.cpu().numpy(), ref.flags), schedule
        assert torch.all(res.stat == 0.0) and torch.all(res.seg_terms[:seg.total] == 0.0), schedule
        assert torch.all(res.n_active == 0), schedule
    stores = tfsc.realisation_stores(gridspec(g), 2, dtype="f32", layout="layer_ci")
    for r in range(2):
        stores[r].pix.copy_(store_from_oracle(d, "f32", layout="layer_ci").pix)
    stores[0].inv_asd.copy_(dev(d["u"]))
    stores[0].tranche_w.copy_(dev(d["wm"]))
    mres = tfsc.bank_statistic_multi(gridspec(g), stores, bt, seg, precision="f32")
    assert np.array_equal(mres.flags.cpu().numpy(), ref.flags)
    assert torch.all(mres.stat == 0.0)


def test_one_tranche_per_segment():
    """N_seg = Nt: every tranche its own segment, so a 64-tranche chunk closes up to 64 segments (the
    segmented reduction's longest walk); FP64 on both schedules against the oracle."""
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    ns = g.n_tranches
    note(f"one tranche per segment (N_seg = {ns})")
    ref = oracle_stat(d, nseg_fixed=ns)
    bt = tfsc.BankTensors.from_host(d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt, nseg_fixed=ns)
    assert seg.total == ns * bt.n
    for schedule, layout in (("thread", "tranche"), ("wave", "layer_ci")):
        res = tfsc.bank_statistic(gridspec(g), store_from_oracle(d, "f64", layout=layout), bt, seg, precision="f64",
                                  schedule=schedule)
        r = rel(res.stat.cpu().numpy(), ref.stat)
        st = res.seg_terms.cpu().numpy()
        note(f"  {schedule}: max rel {r.max():.2e}")
        assert r.max() < 1e-6, schedule
        assert np.max(np.abs(st - ref.seg_terms) / np.maximum(ref.seg_terms, 1.0)) < 1e-6, schedule
        assert np.array_equal(res.flags.cpu().numpy(), ref.flags)


def test_single_channel_channel_interleaved_fp32():
    """C = 1 (TDI A only, the tiny workload) in the channel-interleaved layout, which for one channel is the
    layer-major one: FP32 wave form against the oracle, and equal to the layer-major store bit for bit."""
    tfsc = lib()
    d = tiny_data()
    g = d["grid"]
    note("single channel, channel-interleaved FP32")
    ref = oracle_stat(d)
    bt = tfsc.BankTensors.from_host(d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt, nseg_fixed=8)
    a = tfsc.bank_statistic(gridspec(g), store_from_oracle(d, "f32", layout="layer_ci"), bt, seg, precision="f32",
                            schedule="wave")
    b = tfsc.bank_statistic(gridspec(g), store_from_oracle(d, "f32", layout="layer"), bt, seg, precision="f32",
                            schedule="wave")
    assert torch.equal(a.stat, b.stat)
    r = rel(a.stat.cpu().numpy(), ref.stat)
    note(f"  max rel {r.max():.2e}")
    assert r.max() < 1e-4
    assert int(np.argmax(a.stat.cpu().numpy())) == 256
