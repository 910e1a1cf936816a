"""A caller's orbit table (tfsc_pixels.orbit; Sec. "Outlook": numerical and generic orbits at no extra cost)
through the C ABI.

* tfsc_orbit_positions writes the analytic orbit (against the oracle's positions), and that table fed back
  gives the statistic and the VJP of the built-in orbit bit for bit.
* A rigidly rotated constellation with the sky rotated with it gives the analytic orbit's statistic.
* A perturbed (non-rigid) table against the oracle given the same table.
"""
import math

import numpy as np
import pytest
import torch

import tfsc_inputs as ti
from oracle import o2
from oracle import response as rsp
from oracle import track as otrk

from gpu_common import dev, gridspec, lib, note, rel, small_data, store_from_oracle

pytestmark = pytest.mark.gpu


def _rot_z(tab, a):
    c, s = math.cos(a), math.sin(a)
    out = tab.clone()
    out[:, 0, :] = c * tab[:, 0, :] - s * tab[:, 1, :]
    out[:, 1, :] = s * tab[:, 0, :] + c * tab[:, 1, :]
    return out.contiguous()


def tfsc_store(store, orbit):
    """The same store read with a caller's orbit table."""
    from dataclasses import replace
    return replace(store, orbit=orbit)


def test_analytic_table_is_the_built_in_orbit():
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    grid = gridspec(g)
    tab = tfsc.orbit_positions(grid)
    t = torch.arange(g.n_tranches, dtype=torch.float64) * g.tranche_dur
    ref = rsp.orbits(t).permute(1, 2, 0).numpy()
    err = np.max(np.abs(tab.cpu().numpy() - ref))
    note(f"orbit positions vs the oracle's: max abs {err:.2e} light-seconds (of ~500)")
    assert err < 1e-9
    bt = tfsc.BankTensors.from_host(d["bank"])
    seg = tfsc.segment_layout(grid, bt)
    for dtype, layout, schedule in (("f64", "layer", "wave"), ("f32", "layer_ci", "wave"), ("f32", "tranche", "thread")):
        store = store_from_oracle(d, dtype, layout)
        a = tfsc.bank_statistic(grid, store, bt, seg, precision=dtype, schedule=schedule, want_zn=True)
        b = tfsc.bank_statistic(grid, tfsc_store(store, tab), bt, seg, precision=dtype, schedule=schedule,
                                want_zn=True)
        assert torch.equal(a.stat, b.stat) and torch.equal(a.flags, b.flags), (dtype, schedule)
        if schedule == "wave":
            ones = torch.ones(bt.n, dtype=torch.float64, device="cuda")
            ga = tfsc.statistic_vjp(grid, store, bt, seg, a.seg_zn, g_stat=ones)
            gb = tfsc.statistic_vjp(grid, tfsc_store(store, tab), bt, seg, b.seg_zn, g_stat=ones)
            assert torch.equal(ga, gb)


def test_rotated_constellation_is_the_rotated_sky():
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    grid = gridspec(g)
    ang = 0.83
    tab = _rot_z(tfsc.orbit_positions(grid), ang)
    b = d["bank"]
    br = b.subset(np.arange(len(b)))
    br.phi = b.phi + ang
    bt, btr = tfsc.BankTensors.from_host(b), tfsc.BankTensors.from_host(br)
    seg = tfsc.segment_layout(grid, bt)
    store = store_from_oracle(d, "f64", "layer_ci")
    a = tfsc.bank_statistic(grid, store, bt, seg, precision="f64", schedule="wave")
    r = tfsc.bank_statistic(grid, tfsc_store(store, tab), btr, seg, precision="f64", schedule="wave")
    e = rel(r.stat.cpu().numpy(), a.stat.cpu().numpy())
    note(f"rotated constellation and sky: max rel {e.max():.2e}")
    assert e.max() < 1e-9
    assert torch.equal(a.flags, r.flags)


def test_perturbed_orbit_against_the_oracle():
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    grid = gridspec(g)
    t = torch.arange(g.n_tranches, dtype=torch.float64) * g.tranche_dur
    tab = rsp.orbits(t).permute(1, 2, 0).numpy().copy()
    # non-rigid: spacecraft 1 breathes along z by 0.3 light-seconds over the span, spacecraft 2 lags in x
    tab[1, 2, :] += 0.3 * np.sin(2 * np.pi * np.arange(g.n_tranches) / g.n_tranches)
    tab[2, 0, :] -= 0.2
    b = d["bank"]
    ref = o2.statistic(d["pix"], d["u"], d["wm"], b, g, layout=otrk.Layout(b, g), orbit=tab)
    plain = o2.statistic(d["pix"], d["u"], d["wm"], b, g, layout=otrk.Layout(b, g))
    bt = tfsc.BankTensors.from_host(b)
    seg = tfsc.segment_layout(grid, bt)
    for dtype, layout, tol in (("f64", "layer_ci", 1e-6), ("f32", "layer_ci", 1e-4)):
        store = tfsc_store(store_from_oracle(d, dtype, layout), dev(tab))
        res = tfsc.bank_statistic(grid, store, bt, seg, precision=dtype, schedule="wave")
        e = rel(res.stat.cpu().numpy(), ref.stat)
        moved = rel(plain.stat, ref.stat).max()
        note(f"perturbed orbit {dtype}: max rel vs oracle {e.max():.2e} (the orbit moves Upsilon by {moved:.1e})")
        assert e.max() < tol
        assert moved > 10 * tol
        assert np.array_equal(res.flags.cpu().numpy(), ref.flags)
