"""A bank given in ln Mc (tfsc_bank.ln_mc, the differentiable parameter of the VJP) through the C ABI: the
same results as the bank given in Mc, to the rounding of exp (the device's FP64 exp is within an ulp of the
host's), for the layout, the track, both statistic schedules, the VJP and the follow-up step."""
import math

import numpy as np
import pytest
import torch

from gpu_common import gridspec, lib, note, rel, small_data, store_from_oracle
from oracle import track as otrk

pytestmark = pytest.mark.gpu


def _banks(tfsc, b):
    bt = tfsc.BankTensors.from_host(b)
    # the invalid row (negative mass) has ln Mc = NaN and stays invalid
    with np.errstate(invalid="ignore"):
        ln = torch.as_tensor(np.log(b.mc), device="cuda")
    bl = tfsc.BankTensors(None, bt.eta, bt.f0, bt.cos_theta, bt.phi, bt.psi, bt.cos_iota, ln_mc=ln)
    return bt, bl


def test_ln_mc_bank_gives_the_mc_bank_results():
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    grid = gridspec(g)
    bt, bl = _banks(tfsc, d["bank"])
    sa, sl = tfsc.segment_layout(grid, bt), tfsc.segment_layout(grid, bl)
    assert torch.equal(sa.nseg, sl.nseg)
    ta, tl = tfsc.track(grid, bt), tfsc.track(grid, bl)
    assert torch.equal(ta[..., 3], tl[..., 3])
    assert float(torch.max(torch.abs(ta[..., :3] - tl[..., :3]) / torch.clamp(ta[..., :3].abs(), min=1e-300))) < 1e-12
    for dtype, layout, schedule in (("f64", "layer", "wave"), ("f32", "layer_ci", "wave"), ("f64", "tranche", "thread")):
        store = store_from_oracle(d, dtype, layout)
        a = tfsc.bank_statistic(grid, store, bt, sa, precision=dtype, schedule=schedule, want_zn=True)
        c = tfsc.bank_statistic(grid, store, bl, sl, precision=dtype, schedule=schedule, want_zn=True)
        r = rel(c.stat.cpu().numpy(), a.stat.cpu().numpy())
        note(f"ln Mc bank, {dtype} {schedule}: max rel {r.max():.2e}")
        # exp(ln Mc) may differ from the stored Mc by an ulp, which moves the phase at the end of a long track by
        # up to ~1e-6 rad (the tracks above agree to 1e-12 relative) and Upsilon by a few 1e-8
        assert r.max() < (1e-7 if dtype == "f64" else 1e-5)
        assert torch.equal(a.flags, c.flags)
        if schedule == "wave" and dtype == "f64":
            ones = torch.ones(bt.n, dtype=torch.float64, device="cuda")
            ga = tfsc.statistic_vjp(grid, store, bt, sa, a.seg_zn, g_stat=ones).cpu().numpy()
            gl = tfsc.statistic_vjp(grid, store, bl, sl, c.seg_zn, g_stat=ones).cpu().numpy()
            floor = 1e-3 * np.max(np.abs(ga), axis=0, keepdims=True)
            e = np.abs(gl - ga) / np.maximum(np.abs(ga), floor)
            note(f"  VJP: max rel {e.max():.2e}")
            assert e.max() < 1e-6


def test_ln_mc_bank_processing_order():
    """The processing order of a bank given in ln Mc sorts by the f0 bin and, within a bin, by ln Mc classes
    1/256 of [ln 0.5, ln 500) wide, as for the bank given in Mc."""
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    b = d["bank"]
    bt, bl = _banks(tfsc, b)
    K = g.tranche_len // 2 + 1
    valid = otrk.params_valid(b.mc, b.eta, b.f0, b.cos_theta, b.cos_iota)
    key = np.where(valid, np.clip(np.floor(b.f0 * g.tranche_dur), 0, K - 1), K)
    width = (math.log(500.0) - math.log(0.5)) / 256
    with np.errstate(invalid="ignore"):
        lnmc = np.log(b.mc)
    for bank in (bt, bl):
        order = tfsc.processing_order(gridspec(g), bank).cpu().numpy()
        assert np.array_equal(np.sort(order), np.arange(len(b)))
        assert np.all(np.diff(key[order]) >= 0)
        same = (np.diff(key[order]) == 0) & (key[order][1:] < K)
        assert np.any(same)
        assert np.all(np.diff(lnmc[order])[same] > -width * (1 + 1e-9))


def test_follow_up_step_moves_ln_mc():
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    grid = gridspec(g)
    bt, bl = _banks(tfsc, d["bank"])
    bt = tfsc.BankTensors(*(t.clone() for t in (bt.mc, bt.eta, bt.f0, bt.cos_theta, bt.phi, bt.psi, bt.cos_iota)))
    bl = tfsc.BankTensors(None, bt.eta.clone(), bt.f0.clone(), bt.cos_theta.clone(), bt.phi.clone(), bt.psi.clone(),
                          bt.cos_iota.clone(), ln_mc=bl.ln_mc.clone())
    seg = tfsc.segment_layout(grid, bt)
    store = store_from_oracle(d, "f64", "layer")
    res = tfsc.bank_statistic(grid, store, bt, seg, precision="f64", want_zn=True)
    gp = tfsc.statistic_vjp(grid, store, bt, seg, res.seg_zn, g_stat=torch.ones(bt.n, dtype=torch.float64,
                                                                                   device="cuda"))
    sa = torch.empty((bt.n, 16), dtype=torch.float64, device="cuda")
    sl = torch.empty_like(sa)
    ln0 = bl.ln_mc.clone()
    tfsc.follow_up_step(grid, bt, seg, res.stat, gp, sa, 0.5, 1)
    tfsc.follow_up_step(grid, bl, seg, res.stat, gp, sl, 0.5, 1)
    ok = torch.isfinite(bl.ln_mc)
    moved = (bl.ln_mc[ok] - ln0[ok]).abs().max().item()
    diff = (torch.exp(bl.ln_mc[ok]) - bt.mc[ok]).abs().max().item() / bt.mc[ok].abs().max().item()
    note(f"follow-up step in ln Mc: largest step {moved:.2e}, chirp masses agree to {diff:.1e}")
    assert moved > 0.0 and diff < 1e-12
    assert torch.equal(bl.f0, bt.f0) and torch.equal(bl.phi, bt.phi)
