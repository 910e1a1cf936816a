"""GPU parity of the statistic's vector-Jacobian product against the FP64 oracle's autograd (through the C ABI)."""
import json
import os

import numpy as np
import pytest
import torch

import tfsc_inputs as ti
from oracle import o2
from oracle import track as otrk

from gpu_common import dev, gridspec, lib, note, small_data, store_from_oracle, tiny_data

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _rel_err(g, ref):
    """Per-parameter error of a [n][5] gradient, relative to max(|ref|, 1e-3 x the largest |ref| of that column).

    The floor keeps components that happen to sit near zero (e.g. at a template on the peak) from
    dominating: their absolute error is judged against the gradient scale of the set.
    """
    g, ref = np.asarray(g), np.asarray(ref)
    floor = 1e-3 * np.max(np.abs(ref), axis=0, keepdims=True)
    return np.abs(g - ref) / np.maximum(np.abs(ref), np.maximum(floor, 1e-300))


def _resolution(d, lay):
    """Per-template resolution cells s[n][5]: delta ln Mc = delta f0 / ((5/3) fdot(0) T_obs), delta f0 = 0.1 / T_seg,
    0.05 for cos theta, phi and psi (the follow-up's step scales)."""
    g = d["grid"]
    T = g.n_tranches * g.tranche_dur
    df0 = 0.1 / (T / lay.nseg.astype(np.float64))
    s = np.empty((lay.n, 5))
    s[:, 0] = df0 / ((5.0 / 3.0) * np.abs(lay.fdot0) * T)
    s[:, 1] = df0
    s[:, 2:] = 0.05
    return s


def _cell_err(g, ref, s, ups):
    """Error of the gradient in units of Upsilon per resolution cell: |dg_p| s_p / max(Upsilon, 1)."""
    return np.abs(np.asarray(g) - np.asarray(ref)) * s / np.maximum(np.asarray(ups), 1.0)[:, None]


def _oracle_grads(d, idx, g_seg=None, g_stat=1.0, nseg_fixed=None):
    b = d["bank"]
    lay = otrk.Layout(b, d["grid"], nseg_fixed=nseg_fixed) if nseg_fixed else otrk.Layout(b, d["grid"])
    out = np.zeros((len(idx), 5))
    for r, i in enumerate(idx):
        gs = None
        if g_seg is not None:
            o = lay.seg_offset[i]
            gs = g_seg[o:o + lay.nseg[i]] + g_stat
        elif g_stat != 1.0:
            gs = np.full(lay.nseg[i], g_stat)
        out[r], _ = o2.gradient(d["pix"], d["u"], d["wm"], b, d["grid"], int(i), g_seg=gs, layout=lay)
    return out


def test_vjp_tiny_fp64_matches_oracle_autograd():
    """Tiny workload, FP64 pixels and forward: gradient of Upsilon vs torch float64 autograd of the oracle."""
    tfsc = lib()
    d = tiny_data()
    g = d["grid"]
    idx = np.array([0, 17, 100, 137, 200, 255, 256])
    note(f"vjp tiny fp64, templates {idx.tolist()}")
    bt = tfsc.BankTensors.from_host(d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt, nseg_fixed=8)
    store = store_from_oracle(d, "f64")
    res = tfsc.bank_statistic(gridspec(g), store, bt, seg, precision="f64", schedule="wave", want_zn=True)
    gp = tfsc.statistic_vjp(gridspec(g), store, bt, seg, res.seg_zn,
                            g_stat=torch.ones(bt.n, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    gp = gp.cpu().numpy()[idx]
    ref = _oracle_grads(d, idx)
    err = _rel_err(gp, ref)
    for r, i in enumerate(idx):
        note(f"  #{i}: gpu {np.array2string(gp[r], precision=6)}")
        note(f"       ref {np.array2string(ref[r], precision=6)}  max rel {err[r].max():.2e}")
    assert err.max() < 1e-6


def test_vjp_two_channel_gapped_segment_weights():
    """Two channels, gaps, modulation, adaptive N_seg; random per-segment cotangents plus g_stat; FP64."""
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    b = d["bank"]
    lay = otrk.Layout(b, g)
    rng = np.random.default_rng(5)
    g_seg = rng.normal(size=int(lay.seg_offset[-1]))
    g_stat = 0.5
    ok = np.nonzero((lay.flags & (otrk.FLAG_INVALID | otrk.FLAG_EMPTY)) == 0)[0]
    idx = np.concatenate([ok[:6], ok[-3:]])
    with open(os.path.join(HERE, "golden", "vjp_mp_small.json")) as fh:
        golden = json.load(fh)
    assert golden["g_stat"] == g_stat and golden["g_seg_seed"] == 5
    note(f"vjp 2ch gapped, templates {idx.tolist()}")
    bt = tfsc.BankTensors.from_host(b)
    seg = tfsc.segment_layout(gridspec(g), bt)
    store = store_from_oracle(d, "f64")
    res = tfsc.bank_statistic(gridspec(g), store, bt, seg, precision="f64", schedule="wave", want_zn=True)
    gp = tfsc.statistic_vjp(gridspec(g), store, bt, seg, res.seg_zn,
                            g_stat=torch.full((bt.n,), g_stat, dtype=torch.float64, device="cuda"),
                            g_seg=dev(g_seg))
    gp = gp.cpu().numpy()
    bad = np.nonzero(lay.flags & (otrk.FLAG_INVALID | otrk.FLAG_EMPTY))[0]
    assert np.all(gp[bad] == 0.0)
    ref = _oracle_grads(d, idx, g_seg=g_seg, g_stat=g_stat)
    err = _rel_err(gp[idx], ref)
    cell = _cell_err(gp[idx], ref, _resolution(d, lay)[idx], res.stat.cpu().numpy()[idx])
    for r, i in enumerate(idx):
        note(f"  #{i}: gpu {np.array2string(gp[i], precision=9)}")
        note(f"       ref {np.array2string(ref[r], precision=9)}")
        note(f"       rel {np.array2string(err[r], precision=2)} per cell {cell[r].max():.2e}")
    # Against the 60-digit reference (exact except for the float64 phase rounding that every float64
    # track shares): 1e-6 relative per component.
    for key, row in golden["templates"].items():
        i = int(key)
        ref_mp = np.array(row["grad_f64phase"])
        r_mp = np.abs(gp[i] - ref_mp) / np.abs(ref_mp)
        note(f"  #{i} vs 60-digit reference: rel {np.array2string(r_mp, precision=2)}")
        assert r_mp.max() < 1e-6, i
    # Against float64 autograd of the literal oracle: that oracle loses digits in its derivative at
    # small beta = fdot dT^2 (phases pi (f - f_k)^2 / fdot of 1e6 rad whose derivatives cancel), a few
    # 1e-6 relative at beta ~ 2e-5, so the bar here is looser; per resolution cell it stays tight.
    assert err.max() < 2e-5
    assert cell.max() < 1e-7


@pytest.mark.parametrize("dtype,arith,tol", [("f32", "f64", 1e-4), ("f16", "f64", 5e-3), ("f32", "f32", 1e-4),
                                              ("f16", "f32", 5e-3), ("i16", "f32", 1e-4)])
def test_vjp_reduced_precision_pixels(dtype, arith, tol):
    """FP32 or FP16 pixels with the FP32 forward's (z_n, N_n): error of the FP64 or FP32 VJP against the oracle.

    The bar is in Upsilon units per resolution cell: following the gradient error across one cell moves
    Upsilon by less than tol of itself (the forward's own FP32 bar is 1e-4 relative)."""
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    b = d["bank"]
    lay = otrk.Layout(b, g)
    ok = np.nonzero((lay.flags & (otrk.FLAG_INVALID | otrk.FLAG_EMPTY)) == 0)[0]
    idx = ok[::9][:8]
    note(f"vjp {dtype} pixels, {arith} arithmetic, templates {idx.tolist()}")
    bt = tfsc.BankTensors.from_host(b)
    seg = tfsc.segment_layout(gridspec(g), bt)
    if dtype == "f32":
        store = store_from_oracle(d, "f32")
    else:
        store = tfsc.transform(gridspec(g), dev(d["x"].astype(np.float32)), dev(d["psd"]), dev(d["mu"]),
                               dev(d["keep"]), dtype=dtype)
    res = tfsc.bank_statistic(gridspec(g), store, bt, seg, precision="f32", schedule="wave", want_zn=True)
    gp = tfsc.statistic_vjp(gridspec(g), store, bt, seg, res.seg_zn, precision=arith,
                            g_stat=torch.ones(bt.n, dtype=torch.float64, device="cuda")).cpu().numpy()
    ref = _oracle_grads(d, idx)
    err = _rel_err(gp[idx], ref)
    cell = _cell_err(gp[idx], ref, _resolution(d, lay)[idx], res.stat.cpu().numpy()[idx])
    note(f"  rel: max {err.max():.2e} median {np.median(err):.2e}; per cell: max {cell.max():.2e} "
         f"median {np.median(cell):.2e}")
    for r, i in enumerate(idx):
        note(f"  #{i}: rel {np.array2string(err[r], precision=2)} per cell {np.array2string(cell[r], precision=2)}")
    assert cell.max() < tol


def test_vjp_fp32_arithmetic_against_fp64_on_every_template():
    """The FP32 VJP against the FP64 VJP on the same FP64 store and (z_n, N_n), every template of the gapped,
    modulated two-channel data with random per-segment cotangents: per resolution cell within 1e-5 of
    Upsilon (ten times below the bar against the oracle), invalid and empty templates exactly 0."""
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    b = d["bank"]
    lay = otrk.Layout(b, g)
    note(f"vjp fp32 arithmetic vs fp64, {lay.n} templates")
    rng = np.random.default_rng(17)
    g_seg = rng.normal(size=int(lay.seg_offset[-1]))
    bt = tfsc.BankTensors.from_host(b)
    seg = tfsc.segment_layout(gridspec(g), bt)
    store = store_from_oracle(d, "f64")
    res = tfsc.bank_statistic(gridspec(g), store, bt, seg, precision="f64", schedule="wave", want_zn=True)
    kw = dict(g_stat=torch.full((bt.n,), 0.5, dtype=torch.float64, device="cuda"), g_seg=dev(g_seg))
    g64 = tfsc.statistic_vjp(gridspec(g), store, bt, seg, res.seg_zn, precision="f64", **kw).cpu().numpy()
    g32 = tfsc.statistic_vjp(gridspec(g), store, bt, seg, res.seg_zn, precision="f32", **kw).cpu().numpy()
    bad = (lay.flags & (otrk.FLAG_INVALID | otrk.FLAG_EMPTY)) != 0
    assert np.all(g32[bad] == 0.0)
    ok = ~bad
    cell = _cell_err(g32[ok], g64[ok], _resolution(d, lay)[ok], res.stat.cpu().numpy()[ok])
    err = _rel_err(g32[ok], g64[ok])
    note(f"  per cell: max {cell.max():.2e} median {np.median(cell):.2e}; relative: max {err.max():.2e} "
         f"median {np.median(err):.2e}")
    assert cell.max() < 1e-5


def test_vjp_channel_interleaved_store_equals_layer_major():
    """The VJP reads LAYER_MAJOR_CI pixels at the same values as LAYER_MAJOR ones: same gradients bit for bit."""
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    note("vjp channel-interleaved store")
    bt = tfsc.BankTensors.from_host(d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt)
    out = []
    for layout in ("layer", "layer_ci"):
        store = store_from_oracle(d, "f32", layout=layout)
        res = tfsc.bank_statistic(gridspec(g), store, bt, seg, precision="f32", schedule="wave", want_zn=True)
        out.append(tfsc.statistic_vjp(gridspec(g), store, bt, seg, res.seg_zn,
                                      g_stat=torch.ones(bt.n, dtype=torch.float64, device="cuda")))
    assert torch.equal(out[0], out[1])


def test_autograd_function_uses_the_vjp():
    """TFSCStatistic.backward returns the C-ABI VJP; one gradient-ascent step on the tiny data raises Upsilon."""
    tfsc = lib()
    d = tiny_data()
    g = d["grid"]
    note("autograd function")
    store = store_from_oracle(d, "f64")
    inj = ti.TINY_INJECTION
    n = 4
    ln_mc = torch.full((n,), float(np.log(inj["mc"])), dtype=torch.float64, device="cuda")
    ln_mc += torch.tensor([0.0, 1e-4, -1e-4, 2e-4], dtype=torch.float64, device="cuda")
    f0 = torch.full((n,), inj["f0"], dtype=torch.float64, device="cuda") * (1.0 + torch.tensor(
        [2e-5, 0.0, -2e-5, 1e-5], dtype=torch.float64, device="cuda"))
    ct = torch.full((n,), inj["cos_theta"], dtype=torch.float64, device="cuda")
    ph = torch.full((n,), inj["phi"], dtype=torch.float64, device="cuda")
    ps = torch.full((n,), inj["psi"], dtype=torch.float64, device="cuda")
    fixed = dict(grid=gridspec(g), pixels=store, eta=torch.full((n,), 0.25, dtype=torch.float64, device="cuda"),
                 cos_iota=torch.full((n,), inj["cos_iota"], dtype=torch.float64, device="cuda"), nseg_fixed=8,
                 precision="f64")
    params = [t.clone().requires_grad_(True) for t in (ln_mc, f0, ct, ph, ps)]
    ups = tfsc.TFSCStatistic.apply(*params, fixed)
    grads = torch.autograd.grad(ups.sum(), params)
    # the same through the raw binding (the bank given in ln Mc, as the autograd function passes it)
    bank = tfsc.BankTensors(None, fixed["eta"], f0, ct, ph, ps, fixed["cos_iota"], ln_mc=ln_mc)
    seg = tfsc.segment_layout(fixed["grid"], bank, nseg_fixed=8)
    res = tfsc.bank_statistic(fixed["grid"], store, bank, seg, precision="f64", want_zn=True)
    gp = tfsc.statistic_vjp(fixed["grid"], store, bank, seg, res.seg_zn,
                            g_stat=torch.ones(n, dtype=torch.float64, device="cuda"))
    for p in range(5):
        assert torch.equal(grads[p], gp[:, p])
    # A step along the gradient preconditioned by the statistic's resolution s_p (d_p = eta s_p^2 g_p,
    # first-order gain eta sum s_p^2 g_p^2 = 0.5) raises Upsilon; second-order terms are ~1/Upsilon smaller.
    s = torch.tensor([1.4e-3, 2.5e-7, 0.05, 0.05, 0.05], dtype=torch.float64, device="cuda")
    G = torch.stack(grads, dim=1)
    eta = 0.5 / (s * s * G * G).sum(dim=1)
    newp = [(params[p] + eta * s[p] * s[p] * G[:, p]).detach() for p in range(5)]
    ups2 = tfsc.TFSCStatistic.apply(*newp, fixed)
    note(f"  before {ups.detach().cpu().numpy()}  after {ups2.cpu().numpy()}")
    assert bool((ups2 > ups.detach()).all())


def test_follow_up_raises_upsilon_near_the_injection():
    """Adam follow-up from starts one to two resolution cells off the tiny injection climbs towards it."""
    tfsc = lib()
    d = tiny_data()
    g = d["grid"]
    inj = ti.TINY_INJECTION
    note("follow-up on the tiny injection")
    store = store_from_oracle(d, "f64")
    rng = np.random.default_rng(11)
    n = 16
    b = ti.Bank(mc=inj["mc"] * np.exp(rng.uniform(-2, 2, n) * 1.4e-3), eta=np.full(n, 0.25),
                f0=inj["f0"] + rng.uniform(-2, 2, n) * 2.5e-7, cos_theta=np.full(n, inj["cos_theta"]) + 0.05,
                phi=np.full(n, inj["phi"]) - 0.05, psi=np.full(n, inj["psi"]),
                cos_iota=np.full(n, inj["cos_iota"]), phase=np.zeros(n))
    bt = tfsc.BankTensors.from_host(b)
    first, best, pars = tfsc.follow_up(gridspec(g), store, bt, steps=30, lr_scale=0.5, nseg_fixed=8,
                                       precision="f64")
    first, best = first.cpu().numpy(), best.cpu().numpy()
    exact = tfsc.bank_statistic(gridspec(g), store, tfsc.BankTensors.from_host(ti.tiny_bank().subset([256])),
                                tfsc.segment_layout(gridspec(g), tfsc.BankTensors.from_host(
                                    ti.tiny_bank().subset([256])), nseg_fixed=8), precision="f64").stat.item()
    note(f"  exact {exact:.1f}; start median {np.median(first):.1f}; best median {np.median(best):.1f} "
         f"min gain {np.min(best - first):.2f}")
    assert np.all(best >= first)
    assert np.median(best - first) > 0.0
    assert np.median(best) > 0.9 * exact
    # the caller's bank is untouched
    assert np.array_equal(bt.mc.cpu().numpy(), b.mc)
