"""GPU parity of the statistic path against the FP64 oracle (HIP through the C ABI)."""
import functools

import math

import numpy as np
import pytest
import torch

import tfsc_inputs as ti
from oracle import track as otrk

from gpu_common import dev, gridspec, lib, note, oracle_stat, rel, small_data, store_from_oracle, tiny_data

pytestmark = pytest.mark.gpu


def _bank(tfsc, b):
    return tfsc.BankTensors.from_host(b)


def test_track_bit_exact():
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    b = d["bank"]
    note(f"track bit-exactness, {len(b)} templates x {g.n_tranches} tranches")
    out = tfsc.track(gridspec(g), _bank(tfsc, b)).cpu().numpy()
    lay = otrk.Layout(b, g)
    t = torch.arange(g.n_tranches, dtype=torch.float64) * g.tranche_dur
    checked = 0
    for i in range(len(b)):
        code = out[i, :, 3].astype(np.int64)
        if not lay.valid[i]:
            assert np.all(code == otrk.FLAG_INVALID)
            continue
        first = np.nonzero(code)[0]
        m_end = first[0] if first.size else g.n_tranches
        assert m_end == lay.m_end[i], i
        T = lay.template(i)
        n_ok = int(m_end)
        Phi, f, fdot, _ = T.at(t[:n_ok])
        assert np.array_equal(out[i, :n_ok, 1], f.numpy()), i
        assert np.array_equal(out[i, :n_ok, 2], fdot.numpy()), i
        assert np.array_equal(out[i, :n_ok, 0], Phi.numpy()), i
        # bin index ceil(f dT) therefore agrees bit for bit
        checked += n_ok
    assert checked > 10000


def test_layout_bit_exact():
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    b = d["bank"]
    note("segment layout, rule and fixed")
    for fixed in (0, 7):
        seg = tfsc.segment_layout(gridspec(g), _bank(tfsc, b), nseg_fixed=fixed)
        lay = otrk.Layout(b, g, nseg_fixed=fixed or None) if fixed else otrk.Layout(b, g)
        assert np.array_equal(seg.nseg.cpu().numpy(), lay.nseg)
        assert np.array_equal(seg.seg_offset.cpu().numpy(), lay.seg_offset)


@pytest.mark.parametrize("schedule", ["thread", "wave"])
def test_tiny_fp64_matches_oracle(schedule):
    """Tiny workload (257 templates incl. the exact one), FP64 pixels and arithmetic: 1e-6."""
    tfsc = lib()
    d = tiny_data()
    g = d["grid"]
    note(f"tiny fp64 {schedule}")
    ref = oracle_stat(d, want_zn=True)
    bt = _bank(tfsc, d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt, nseg_fixed=8)
    res = tfsc.bank_statistic(gridspec(g), store_from_oracle(d, "f64"), bt, seg, precision="f64", schedule=schedule,
                              want_zn=True)
    torch.cuda.synchronize()
    stat = res.stat.cpu().numpy()
    assert rel(stat, ref.stat).max() < 1e-6
    assert np.array_equal(res.flags.cpu().numpy(), ref.flags)
    assert np.max(np.abs(res.seg_terms.cpu().numpy() - ref.seg_terms) / np.maximum(ref.seg_terms, 1.0)) < 1e-6
    zn = res.seg_zn.cpu().numpy()
    # (z_n, N_n) come out with the exact weight normalisation 2^-e, e = exponent of max u_k
    sc = 2.0 ** (-np.frexp(np.max(d["u"]))[1])
    assert np.allclose(zn[:, 2], ref.seg_zn[:, 2] * sc * sc, rtol=1e-9)
    assert np.allclose(zn[:, 0], ref.seg_zn[:, 0] * sc, rtol=1e-6, atol=1e-9 * np.abs(ref.seg_zn[:, 0] * sc).max())
    # the injected template ranks first
    assert int(np.argmax(stat)) == 256
    note(f"tiny fp64 {schedule}: max rel {rel(stat, ref.stat).max():.2e}, exact-template stat {stat[256]:.1f}")


@pytest.mark.parametrize("schedule", ["thread", "wave"])
@pytest.mark.parametrize("precision,pixdt,tol", [("f64", "f64", 1e-6), ("f64", "f32", 1e-5), ("f32", "f32", 1e-4)])
def test_two_channel_gapped_matches_oracle(schedule, precision, pixdt, tol):
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    note(f"2ch gapped {schedule} {precision} pixels {pixdt}")
    ref = oracle_stat(d)
    bt = _bank(tfsc, d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt)
    res = tfsc.bank_statistic(gridspec(g), store_from_oracle(d, pixdt), bt, seg, precision=precision,
                              schedule=schedule)
    stat = res.stat.cpu().numpy()
    r = rel(stat, ref.stat)
    note(f"  max rel {r.max():.2e} median {np.median(r):.2e}")
    assert r.max() < tol
    assert np.array_equal(res.flags.cpu().numpy(), ref.flags)
    seg_ref = ref.seg_terms
    assert np.max(np.abs(res.seg_terms.cpu().numpy() - seg_ref) / np.maximum(seg_ref, 1.0)) < 10 * tol


def test_tranche_major_thread_schedule():
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    note("tranche-major layout, thread schedule")
    ref = oracle_stat(d)
    bt = _bank(tfsc, d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt)
    res = tfsc.bank_statistic(gridspec(g), store_from_oracle(d, "f32", layout="tranche"), bt, seg, precision="f32",
                              schedule="thread")
    assert rel(res.stat.cpu().numpy(), ref.stat).max() < 1e-4


@pytest.mark.parametrize("schedule", ["thread", "wave"])
@pytest.mark.parametrize("precision,pixdt", [("f64", "f64"), ("f64", "f32"), ("f32", "f32")])
def test_channel_interleaved_layout_equals_layer_major(schedule, precision, pixdt):
    """LAYER_MAJOR_CI holds the pixels of LAYER_MAJOR with the channels of a (bin, tranche) cell
    adjacent; the arithmetic and its order do not change, so every output is the same bit for bit."""
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    note(f"channel-interleaved store, {schedule} {precision} pixels {pixdt}")
    bt = _bank(tfsc, d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt)
    a = tfsc.bank_statistic(gridspec(g), store_from_oracle(d, pixdt), bt, seg, precision=precision,
                            schedule=schedule)
    ci = store_from_oracle(d, pixdt, layout="layer_ci")
    assert tuple(ci.pix.shape) == (g.tranche_len // 2 + 1, g.n_tranches, g.n_channels, 2)
    b = tfsc.bank_statistic(gridspec(g), ci, bt, seg, precision=precision, schedule=schedule)
    assert torch.equal(a.stat, b.stat) and torch.equal(a.flags, b.flags) and torch.equal(a.seg_terms, b.seg_terms)
    ref = oracle_stat(d)
    assert rel(b.stat.cpu().numpy(), ref.stat).max() < (1e-4 if precision == "f32" else 1e-5)


def _low_bank():
    """Templates starting at 2-15 frequency bins, so the 21-bin window of the first tranches reaches
    below the DC bin; the chirp carries most of them across bin 10 within the observation."""
    return ti.random_bank(256, 7, mc_range=(5.0, 100.0), f0_range=(0.0008, 0.006), eta=None, stream=31)


@functools.lru_cache(maxsize=1)
def _low_reference():
    """Oracle values for the low bank, and 30-digit values (with the float64 phase rounding that every
    float64 track shares) for its four templates of smallest chirp rate.  At such small beta = fdot dT^2
    the float64 oracle's literal Fresnel form loses digits (1.9e-6 relative against the 30-digit value
    for these templates), so the FP64 path is judged against the 30-digit values there."""
    from oracle import o2_mp
    d = small_data()
    b = _low_bank()
    ref = oracle_stat(d, bank=b)
    chirp = b.mc ** (5.0 / 3.0) * b.f0 ** (11.0 / 3.0)
    idx = np.argsort(chirp)[:4]
    mp = np.array([o2_mp.statistic(d["pix"], d["u"], d["wm"], b, d["grid"], int(i), dps=30, float64_phase=True)
                   for i in idx])
    return ref, idx, mp


@pytest.mark.parametrize("layout", ["layer", "layer_ci"])
@pytest.mark.parametrize("precision,pixdt,tol", [("f64", "f64", 1e-6), ("f32", "f32", 1e-4)])
def test_low_frequency_templates_match_oracle(layout, precision, pixdt, tol):
    """The WAVE schedule's path for waves with a lane below bin 10, and the thread schedule, against
    the oracle: FP32 at 1e-4; FP64 at 1e-6 against the 30-digit values of the smallest-beta templates
    and at 3e-6 against the float64 oracle elsewhere (the oracle's own loss at small beta)."""
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    b = _low_bank()
    assert np.sum(b.f0 * g.tranche_dur < 9.0) > 64
    note(f"low-frequency templates, {layout} {precision}")
    ref, idx, mp = _low_reference()
    bt = _bank(tfsc, b)
    seg = tfsc.segment_layout(gridspec(g), bt)
    st = store_from_oracle(d, pixdt, layout=layout)
    tol_oracle = tol if precision == "f32" else 3e-6
    for schedule in ("thread", "wave"):
        res = tfsc.bank_statistic(gridspec(g), st, bt, seg, precision=precision, schedule=schedule)
        s = res.stat.cpu().numpy()
        r = rel(s, ref.stat)
        r_mp = rel(s[idx], mp)
        note(f"  {schedule}: max rel {r.max():.2e} vs oracle; smallest-beta templates {r_mp.max():.2e} vs 30 digits "
             f"(oracle {rel(ref.stat[idx], mp).max():.2e})")
        assert r.max() < tol_oracle, schedule
        assert r_mp.max() < tol, schedule
        assert np.array_equal(res.flags.cpu().numpy(), ref.flags)
        assert np.max(np.abs(res.seg_terms.cpu().numpy() - ref.seg_terms) / np.maximum(ref.seg_terms, 1.0)) < 10 * tol_oracle


def test_processing_order_does_not_change_results():
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    bt = _bank(tfsc, d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt)
    store = store_from_oracle(d, "f32")
    a = tfsc.bank_statistic(gridspec(g), store, bt, seg, precision="f32", schedule="wave")
    perm = torch.randperm(bt.n, generator=torch.Generator().manual_seed(3)).to(torch.int32).cuda()
    b = tfsc.bank_statistic(gridspec(g), store, bt, seg, precision="f32", schedule="wave", order=perm)
    c = tfsc.bank_statistic(gridspec(g), store, bt, seg, precision="f32", schedule="wave", block_waves=2,
                            groups_per_cu=3)
    assert torch.equal(a.stat, b.stat) and torch.equal(a.stat, c.stat)
    assert torch.equal(a.seg_terms, b.seg_terms)


def test_empty_bank_and_errors():
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    b = d["bank"].subset(np.arange(0))
    bt = _bank(tfsc, b)
    seg = tfsc.segment_layout(gridspec(g), bt)
    assert seg.total == 0
    res = tfsc.bank_statistic(gridspec(g), store_from_oracle(d, "f32"), bt, seg, precision="f32")
    assert res.stat.numel() == 0
    with pytest.raises(tfsc.TfscError):
        tfsc.bank_statistic(gridspec(g), store_from_oracle(d, "f32", layout="tranche"), _bank(tfsc, d["bank"]),
                            tfsc.segment_layout(gridspec(g), _bank(tfsc, d["bank"])), precision="f32", schedule="wave")
    with pytest.raises(tfsc.TfscError):
        tfsc.bank_statistic(gridspec(g), store_from_oracle(d, "f64"), _bank(tfsc, d["bank"]),
                            tfsc.segment_layout(gridspec(g), _bank(tfsc, d["bank"])), precision="f32")


@pytest.mark.parametrize("layout", ["layer", "layer_ci"])
@pytest.mark.parametrize("dtype,tol", [("f16", 2e-3), ("bf16", 2e-2), ("i16", 1e-4)])
def test_16bit_store_error_against_oracle(dtype, tol, layout):
    """16-bit pixels with a per-layer FP32 scale, FP32 arithmetic: error of Upsilon vs the FP64 oracle (the
    int16 fixed-point store is held to the 1e-4 bar of the FP32 form)."""
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    note(f"16-bit store {dtype} {layout}")
    x32 = d["x"].astype(np.float32)
    from oracle import transform as otf
    ref_pix, u, wm = otf.transform(x32.astype(np.float64), g, d["psd"], d["mu"], d["keep"], 0.1, "rfft")
    from oracle import cpu as ocpu
    ref = ocpu.statistic(ref_pix, u, wm, d["bank"], g)
    st = tfsc.transform(gridspec(g), dev(x32), dev(d["psd"]), dev(d["mu"]), dev(d["keep"]), dtype=dtype, layout=layout)
    bt = _bank(tfsc, d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt)
    res = tfsc.bank_statistic(gridspec(g), st, bt, seg, precision="f32", schedule="wave")
    r = rel(res.stat.cpu().numpy(), ref.stat)
    note(f"  {dtype}: max rel {r.max():.2e} median {np.median(r):.2e} p99 {np.quantile(r, 0.99):.2e}")
    assert r.max() < tol
    assert np.array_equal(res.flags.cpu().numpy(), ref.flags)


def test_device_processing_order():
    """tfsc_processing_order: a permutation sorted by the f0 bin (invalid last) and, within a bin, by classes of
    ln Mc 1/256 of [ln 0.5, ln 500) wide; results do not depend on it."""
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    b = d["bank"]
    note("device processing order")
    bt = _bank(tfsc, b)
    order = tfsc.processing_order(gridspec(g), bt).cpu().numpy()
    assert np.array_equal(np.sort(order), np.arange(len(b)))
    valid = otrk.params_valid(b.mc, b.eta, b.f0, b.cos_theta, b.cos_iota)
    K = g.tranche_len // 2 + 1
    key = np.where(valid, np.clip(np.floor(b.f0 * g.tranche_dur), 0, K - 1), K)
    assert np.all(np.diff(key[order]) >= 0)
    # within a bin, ln Mc never falls by a class width or more from one template to the next
    width = (math.log(500.0) - math.log(0.5)) / 256
    lnmc = np.log(b.mc)[order]
    same = (np.diff(key[order]) == 0) & (key[order][1:] < K)
    assert np.all(np.diff(lnmc)[same] > -width * (1 + 1e-9))
    assert np.any(same)
    seg = tfsc.segment_layout(gridspec(g), bt)
    store = store_from_oracle(d, "f32")
    a = tfsc.bank_statistic(gridspec(g), store, bt, seg, precision="f32", schedule="wave")
    c = tfsc.bank_statistic(gridspec(g), store, bt, seg, precision="f32", schedule="wave",
                            order=torch.from_numpy(order).cuda())
    assert torch.equal(a.stat, c.stat) and torch.equal(a.flags, c.flags)
