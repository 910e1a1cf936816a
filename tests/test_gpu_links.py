"""A caller's link light times (tfsc_pixels.links; Sec. "Outlook": varying arm lengths and point-ahead light
times of numerical orbits) through the C ABI, against the oracle (``oracle.response``'s unequal-arm form).

* tfsc_link_lengths: |p_r - p_s| of the analytic orbit and of a caller's table, against the oracle's.
* Six equal light times L on an exactly equilateral orbit give the equal-arm statistic.
* Unequal, direction-dependent light times on the analytic orbit and on a perturbed table: both schedules,
  FP64 and FP32, two and three channels, against the oracle given the same table; flags equal.
* Second-generation TDI on the same geometry against the oracle's.
* The calls that do not take the table refuse it.
"""
import functools
import math

import numpy as np
import pytest
import torch

import tfsc_inputs as ti
from oracle import o2
from oracle import response as rsp
from oracle import track as otrk
from oracle import transform as otf

from gpu_common import dev, gridspec, lib, note, rel, small_data, store_from_oracle

pytestmark = pytest.mark.gpu


def _subset(n):
    # every third template and the invalid, empty and face-on rows of small_data's bank
    return sorted(set(range(0, n, 3)) | {3, 5, 7, 9})


def _links_table(g, seed, spread=0.05):
    """Light times that differ between the arms and between the two directions of an arm and drift over the
    span (seconds, [6][Nt])."""
    rng = np.random.default_rng(seed)
    base = rsp.L_S * (1.0 + spread * rng.uniform(-1.0, 1.0, size=6))
    drift = 0.01 * rsp.L_S * np.sin(2.0 * math.pi * np.arange(g.n_tranches) / g.n_tranches)
    return np.ascontiguousarray(base[:, None] + drift[None, :] * np.array([1, -1, 0.5, 1, -1, 0.5])[:, None])


def _equilateral_table(g):
    t = np.arange(g.n_tranches) * g.tranche_dur
    p = rsp.orbits(torch.as_tensor(t, dtype=torch.float64))  # [Nt, 3, 3]
    c = p.mean(dim=1, keepdim=True)
    e1 = p[:, 0] - c[:, 0]
    e1 = e1 / torch.linalg.norm(e1, dim=-1, keepdim=True)
    nrm = torch.linalg.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
    e2 = torch.linalg.cross(nrm / torch.linalg.norm(nrm, dim=-1, keepdim=True), e1)
    rad = rsp.L_S / math.sqrt(3.0)
    q = torch.stack([c[:, 0] + rad * (math.cos(b) * e1 + math.sin(b) * e2)
                     for b in (0.0, 2.0 * math.pi / 3.0, 4.0 * math.pi / 3.0)], dim=1)
    return np.ascontiguousarray(q.permute(1, 2, 0).numpy())  # [3][3][Nt]


def _with(store, orbit=None, links=None):
    from dataclasses import replace
    return replace(store, orbit=orbit, links=links)


@functools.lru_cache(maxsize=2)
def _three_channel_data():
    g = ti.custom_grid(3, 512, 400, dt=5.0, modulated=True, gapped=True, cfg_id=27)
    psd, mu, keep = ti.psd_on_bins(g), ti.tranche_psd_scale(g), ti.tranche_keep(g)
    pix, u, wm = otf.transform(ti.noise(g), g, psd, mu, keep, 0.1, "rfft")
    b = ti.random_bank(24, 27, mc_range=(5.0, 60.0), f0_range=(0.004, 0.06), eta=None, stream=71)
    return dict(grid=g, pix=pix, u=u, wm=wm, bank=b)


def test_link_lengths_against_the_oracle():
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    grid = gridspec(g)
    t = torch.arange(g.n_tranches, dtype=torch.float64) * g.tranche_dur
    ref = rsp.link_lengths(rsp.orbits(t)).T.numpy()
    got = tfsc.link_lengths(grid).cpu().numpy()
    note(f"analytic orbit: link light times {got.min():.6f}..{got.max():.6f} s, max abs vs oracle "
         f"{np.max(np.abs(got - ref)):.1e}")
    assert np.max(np.abs(got - ref)) < 1e-9
    tab = _equilateral_table(g)
    tab[1, 2, :] += 0.2  # spacecraft 1 lifted out of the plane by 0.2 light-seconds
    ref = rsp.link_lengths(torch.as_tensor(tab).permute(2, 0, 1)).T.numpy()
    got = tfsc.link_lengths(grid, dev(tab)).cpu().numpy()
    assert np.max(np.abs(got - ref)) < 1e-9
    assert np.array_equal(got[:3], got[3:])


@pytest.mark.parametrize("dtype,schedule,tol", [("f64", "wave", 1e-9), ("f64", "thread", 1e-9),
                                                 ("f32", "wave", 2e-5)])
def test_equal_links_on_an_equilateral_orbit_are_the_equal_arm_statistic(dtype, schedule, tol):
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    grid = gridspec(g)
    tab = dev(_equilateral_table(g))
    bt = tfsc.BankTensors.from_host(d["bank"])
    seg = tfsc.segment_layout(grid, bt)
    store = store_from_oracle(d, dtype, "layer_ci")
    a = tfsc.bank_statistic(grid, _with(store, tab), bt, seg, precision=dtype, schedule=schedule)
    lk = torch.full((6, g.n_tranches), rsp.L_S, dtype=torch.float64, device="cuda")
    b = tfsc.bank_statistic(grid, _with(store, tab, lk), bt, seg, precision=dtype, schedule=schedule)
    r = rel(b.stat.cpu().numpy(), a.stat.cpu().numpy())
    note(f"equal links, {dtype} {schedule}: max rel vs the equal-arm kernel {r.max():.2e}")
    assert r.max() < tol
    assert torch.equal(a.flags, b.flags)


@pytest.mark.parametrize("dtype,layout,schedule,tol", [("f64", "layer", "wave", 1e-6), ("f64", "layer_ci", "wave", 1e-6),
                                                        ("f64", "tranche", "thread", 1e-6),
                                                        ("f32", "layer_ci", "wave", 1e-4),
                                                        ("f32", "layer", "thread", 1e-4)])
def test_unequal_links_against_the_oracle(dtype, layout, schedule, tol):
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    grid = gridspec(g)
    b = d["bank"]
    idx = _subset(len(b))
    links = _links_table(g, 3)
    ref = o2.statistic(d["pix"], d["u"], d["wm"], b, g, layout=otrk.Layout(b, g), idx=idx, links=links)
    plain = o2.statistic(d["pix"], d["u"], d["wm"], b, g, layout=otrk.Layout(b, g), idx=idx)
    bt = tfsc.BankTensors.from_host(b)
    seg = tfsc.segment_layout(grid, bt)
    store = _with(store_from_oracle(d, dtype, layout), None, dev(links))
    res = tfsc.bank_statistic(grid, store, bt, seg, precision=dtype, schedule=schedule, want_zn=True)
    s = res.stat.cpu().numpy()[idx]
    e = rel(s, ref.stat[idx])
    moved = rel(plain.stat[idx], ref.stat[idx]).max()
    note(f"unequal links {dtype} {layout} {schedule}: max rel vs oracle {e.max():.2e} (the links move Upsilon by "
         f"{moved:.1e})")
    assert e.max() < tol
    assert moved > 10 * tol
    assert np.array_equal(res.flags.cpu().numpy()[idx], ref.flags[idx])


def test_unequal_links_on_a_caller_orbit():
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    grid = gridspec(g)
    b = d["bank"]
    idx = _subset(len(b))
    t = torch.arange(g.n_tranches, dtype=torch.float64) * g.tranche_dur
    tab = rsp.orbits(t).permute(1, 2, 0).numpy().copy()
    tab[2, 0, :] -= 0.3
    tab[0, 2, :] += 0.2 * np.cos(2 * np.pi * np.arange(g.n_tranches) / g.n_tranches)
    links = rsp.link_lengths(torch.as_tensor(tab).permute(2, 0, 1)).T.numpy().copy()
    links[3:] *= 1.0 + 2e-3  # the reverse links a little longer (a point-ahead difference)
    ref = o2.statistic(d["pix"], d["u"], d["wm"], b, g, layout=otrk.Layout(b, g), idx=idx, orbit=tab, links=links)
    bt = tfsc.BankTensors.from_host(b)
    seg = tfsc.segment_layout(grid, bt)
    for dtype, tol in (("f64", 1e-6), ("f32", 1e-4)):
        store = _with(store_from_oracle(d, dtype, "layer_ci"), dev(tab), dev(np.ascontiguousarray(links)))
        res = tfsc.bank_statistic(grid, store, bt, seg, precision=dtype, schedule="wave")
        e = rel(res.stat.cpu().numpy()[idx], ref.stat[idx])
        note(f"caller orbit + links {dtype}: max rel vs oracle {e.max():.2e}")
        assert e.max() < tol
        assert np.array_equal(res.flags.cpu().numpy()[idx], ref.flags[idx])


def test_three_channels_with_links():
    tfsc = lib()
    d = _three_channel_data()
    g = d["grid"]
    grid = gridspec(g)
    b = d["bank"]
    links = _links_table(g, 9)
    ref = o2.statistic(d["pix"], d["u"], d["wm"], b, g, links=links)
    bt = tfsc.BankTensors.from_host(b)
    seg = tfsc.segment_layout(grid, bt)
    for dtype, schedule, tol in (("f64", "wave", 1e-6), ("f32", "wave", 1e-4), ("f64", "thread", 1e-6)):
        store = _with(tfsc.PixelStore.from_complex(dev(d["pix"]), dev(d["u"]), dev(d["wm"]), dtype=dtype,
                                                   layout="layer_ci"), None, dev(links))
        res = tfsc.bank_statistic(grid, store, bt, seg, precision=dtype, schedule=schedule)
        e = rel(res.stat.cpu().numpy(), ref.stat)
        note(f"A + E + T with links, {dtype} {schedule}: max rel vs oracle {e.max():.2e}")
        assert e.max() < tol
        assert np.array_equal(res.flags.cpu().numpy(), ref.flags)


@pytest.mark.parametrize("dtype,schedule,tol", [("f64", "wave", 1e-6), ("f64", "thread", 1e-6), ("f32", "wave", 1e-4)])
def test_second_generation_against_the_oracle(dtype, schedule, tol):
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    grid = gridspec(g)
    b = d["bank"]
    idx = _subset(len(b))
    links = _links_table(g, 13)
    ref = o2.statistic(d["pix"], d["u"], d["wm"], b, g, layout=otrk.Layout(b, g), idx=idx, links=links, generation=2)
    first = o2.statistic(d["pix"], d["u"], d["wm"], b, g, layout=otrk.Layout(b, g), idx=idx, links=links)
    bt = tfsc.BankTensors.from_host(b)
    seg = tfsc.segment_layout(grid, bt)
    store = store_from_oracle(d, dtype, "layer_ci")
    from dataclasses import replace
    store = replace(store, links=dev(links), tdi_generation=2)
    res = tfsc.bank_statistic(grid, store, bt, seg, precision=dtype, schedule=schedule)
    e = rel(res.stat.cpu().numpy()[idx], ref.stat[idx])
    moved = rel(first.stat[idx], ref.stat[idx]).max()
    note(f"second-generation TDI, unequal links, {dtype} {schedule}: max rel vs oracle {e.max():.2e} (the "
         f"generation moves Upsilon by {moved:.1e})")
    assert e.max() < tol
    assert moved > 10 * tol
    assert np.array_equal(res.flags.cpu().numpy()[idx], ref.flags[idx])


def test_calls_without_the_unequal_arm_response_refuse_links():
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    grid = gridspec(g)
    bt = tfsc.BankTensors.from_host(d["bank"])
    seg = tfsc.segment_layout(grid, bt)
    lk = torch.full((6, g.n_tranches), rsp.L_S, dtype=torch.float64, device="cuda")
    store = _with(store_from_oracle(d, "f64", "layer_ci"), None, lk)
    a = tfsc.bank_statistic(grid, store, bt, seg, precision="f64", schedule="wave", want_zn=True)
    with pytest.raises(tfsc.TfscError):
        tfsc.statistic_vjp(grid, store, bt, seg, a.seg_zn, g_stat=torch.ones(bt.n, dtype=torch.float64,
                                                                             device="cuda"))
    with pytest.raises(tfsc.TfscError):
        tfsc.bank_statistic_harmonics(grid, store, bt, seg, [2], torch.ones((bt.n, 1), dtype=torch.complex128,
                                                                           device="cuda"), precision="f64")
    with pytest.raises(tfsc.TfscError):
        tfsc.bank_statistic(grid, store, bt, seg, precision="f64", schedule="wave", fresnel="accurate")
