"""Parity at the full two-year A+E size (Nt = 6144 tranches of 2048 samples, gaps, modulated PSD).

The bank is a random slice of the full-size workload's bank plus its exact-parameter templates;
the oracle evaluates a sample of them one by one on the CPU from its own transform of the same data.
"""
import functools

import numpy as np
import pytest
import torch

import tfsc_inputs as ti
from oracle import cpu as ocpu
from oracle import transform as otf

from gpu_common import dev, gridspec, lib, note, rel

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=1)
def full_data():
    g = ti.FULL
    note("full-size data: noise, gaps, modulation")
    x = (ti.noise(g) * ti.sample_keep_mask(g)[None, :]).astype(np.float32)
    psd = ti.psd_on_bins(g)
    mu, keep = ti.tranche_psd_scale(g), ti.tranche_keep(g)
    pix, u, wm = otf.transform(x.astype(np.float64), g, psd, mu, keep, 0.1, "rfft")
    full = ti.full_bank(200_000)
    idx = np.concatenate([np.arange(200_000, 200_020), ti.subsample_indices(200_000, 1004, cfg_id=11)])
    bank = full.subset(idx)
    return dict(grid=g, x=x, psd=psd, mu=mu, keep=keep, pix=pix, u=u, wm=wm, bank=bank)


@pytest.mark.parametrize("precision,source,schedule,layout", [("f32", "gpu", "wave", "layer_ci"),
                                                              ("f32", "oracle", "wave", "layer"),
                                                              ("f64", "oracle", "wave", "layer_ci"),
                                                              ("f32", "gpu", "thread", "tranche"),
                                                              ("f64", "oracle", "thread", "tranche")])
def test_full_size_sampled_parity(precision, source, schedule, layout):
    tfsc = lib()
    d = full_data()
    g = d["grid"]
    bt = tfsc.BankTensors.from_host(d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt)
    if source == "gpu":
        note(f"full size: GPU transform (f32, {layout}) -> {schedule} statistic ({precision})")
        st = tfsc.transform(gridspec(g), dev(d["x"]), dev(d["psd"]), dev(d["mu"]), dev(d["keep"]), dtype="f32",
                            layout=layout)
    else:
        note(f"full size: oracle pixels stored {precision} ({layout}) -> {schedule} statistic ({precision})")
        st = tfsc.PixelStore.from_complex(dev(d["pix"]), dev(d["u"]), dev(d["wm"]), dtype=precision, layout=layout)
    tol = 1e-4 if precision == "f32" else 1e-6
    res = tfsc.bank_statistic(gridspec(g), st, bt, seg, precision=precision, schedule=schedule)
    stat = res.stat.cpu().numpy()
    flags = res.flags.cpu().numpy()
    sample = np.concatenate([np.arange(20), np.arange(20, len(d["bank"]), 16)])
    ref = ocpu.statistic(d["pix"], d["u"], d["wm"], d["bank"].subset(sample), g)
    r = rel(stat[sample], ref.stat)
    note(f"  {precision}: {sample.size} sampled templates, max rel {r.max():.2e} median {np.median(r):.2e}")
    b = d["bank"]
    for w in np.argsort(r)[-4:]:
        i = sample[w]
        note(f"    worst: idx {i} rel {r[w]:.2e} stat {stat[i]:.3f} ref {ref.stat[w]:.3f} mc {b.mc[i]:.2f} "
             f"f0 {b.f0[i]:.5f} nseg {ref.nseg[w]} m_end {ref.m_end[w]} flags {ref.flags[w]}")
    assert r.max() < tol
    assert np.array_equal(flags[sample], ref.flags)
    seg_off = seg.seg_offset.cpu().numpy()
    assert np.array_equal(np.diff(seg_off)[sample], ref.nseg)
    assert set(np.unique(np.diff(seg_off))) <= {16, 32, 64, 128, 256}


def test_whole_bank_fp32_forms_against_fp64_path():
    """All 1,000,020 templates: both FP32 forms against the FP64 path (itself within 2e-9 of the oracle
    on the sampled templates above), in the bench's configuration."""
    tfsc = lib()
    g = ti.FULL
    note("whole bank: FP32 wave and thread forms vs the FP64 path")
    x = ti.noise(g) * ti.sample_keep_mask(g)[None, :]
    psd, mu, keep = ti.psd_on_bins(g), ti.tranche_psd_scale(g), ti.tranche_keep(g)
    bank_h = ti.full_bank(1_000_000)
    bt = tfsc.BankTensors.from_host(bank_h)
    grid = gridspec(g)
    seg = tfsc.segment_layout(grid, bt)
    order = tfsc.processing_order(grid, bt)
    st64 = tfsc.transform(grid, dev(x), dev(psd), dev(mu), dev(keep), dtype="f64")
    ref = tfsc.bank_statistic(grid, st64, bt, seg, precision="f64", schedule="wave", order=order).stat
    ref = ref.cpu().numpy()
    del st64
    x32 = dev(x.astype(np.float32))
    for schedule, layout in (("wave", "layer_ci"), ("thread", "tranche")):
        st = tfsc.transform(grid, x32, dev(psd), dev(mu), dev(keep), dtype="f32", layout=layout)
        s = tfsc.bank_statistic(grid, st, bt, seg, precision="f32", schedule=schedule,
                                order=order if schedule == "wave" else None).stat.cpu().numpy()
        r = rel(s, ref)
        w = np.argsort(r)[-3:]
        note(f"  {schedule}: max rel {r.max():.2e}  p99.99 {np.quantile(r, 0.9999):.2e}  median {np.median(r):.2e}")
        for i in w:
            note(f"    worst: idx {i} rel {r[i]:.2e} stat {s[i]:.3f} fp64 {ref[i]:.3f} mc {bank_h.mc[i]:.2f} "
                 f"f0 {bank_h.f0[i]:.5f}")
        assert r.max() < 1e-4
        del st
