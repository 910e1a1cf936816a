"""Precision form at the full size: FP32, FP16, BF16 and int16 fixed-point pixel stores against the FP64 oracle.

Workload: the full-size data (2-yr A+E, gaps, modulated PSD) with the 20 injections of the full-size
configuration added in the pixel domain (the oracle's own template pixels, phase-shifted and scaled
to their target SNR), and a 10,000-template subsample of the full-size bank (the first indices of a
seeded permutation, always including the 20 exact-parameter templates).  The FP16 and BF16 stores hold
the oracle's pixels divided by a per-layer FP32 scale (the layer's largest component magnitude); the
int16 store holds the nearest integers to the pixels divided by that magnitude / 32767.
"""
import functools

import numpy as np
import pytest
import torch

import tfsc_inputs as ti
from oracle import cpu as ocpu
from oracle import o2
from oracle import track as otrk
from oracle import transform as otf

from gpu_common import dev, full_injected, gridspec, lib, note

pytestmark = pytest.mark.gpu

N_FULL = 1_000_000


@functools.lru_cache(maxsize=1)
def data():
    d = dict(full_injected())
    g = d["grid"]
    bank = ti.full_bank(N_FULL)
    idx = ti.subsample_indices(len(bank), 10_000, must_include=np.arange(N_FULL, N_FULL + 20), cfg_id=13)
    sub = bank.subset(idx)
    note("precision data: FP64 oracle on the 10,000-template subsample")
    d["ref"] = ocpu.statistic(d["pix"], d["u"], d["wm"], sub, g)
    d["bank"] = sub
    return d


def _store(tfsc, d, dtype):
    if dtype in ("f64", "f32"):
        return tfsc.PixelStore.from_complex(dev(d["pix"]), dev(d["u"]), dev(d["wm"]), dtype=dtype)
    pix = d["pix"]
    scale = np.maximum(np.abs(pix.real), np.abs(pix.imag)).max(axis=2).astype(np.float32)  # [C][K]
    if dtype == "i16":
        step = (scale.astype(np.float64) / 32767.0).astype(np.float32)
        s = np.where(step > 0, step, 1.0).astype(np.float64)[:, :, None]
        q = np.clip(np.rint(np.stack([pix.real / s, pix.imag / s], axis=-1)), -32767, 32767).astype(np.int16)
        return tfsc.PixelStore(torch.from_numpy(np.ascontiguousarray(q)).cuda(), dev(d["u"]), dev(d["wm"]), dtype,
                               "layer", dev(step))
    safe = np.where(scale > 0, scale, 1.0).astype(np.float64)
    q = np.stack([pix.real / safe[:, :, None], pix.imag / safe[:, :, None]], axis=-1)
    tdt = torch.float16 if dtype == "f16" else torch.bfloat16
    t = torch.from_numpy(np.ascontiguousarray(q)).to(tdt).cuda()
    return tfsc.PixelStore(t, dev(d["u"]), dev(d["wm"]), dtype, "layer", dev(scale))


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-4), ("f16", 2e-3), ("bf16", 2e-2), ("i16", 1e-4)])
def test_precision_forms_against_oracle(dtype, tol):
    tfsc = lib()
    d = data()
    g = d["grid"]
    bt = tfsc.BankTensors.from_host(d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt)
    res = tfsc.bank_statistic(gridspec(g), _store(tfsc, d, dtype), bt, seg, precision="f32", schedule="wave",
                              order=tfsc.processing_order(gridspec(g), bt))
    stat = res.stat.cpu().numpy()
    ref = d["ref"].stat
    r = np.abs(stat - ref) / np.maximum(np.abs(ref), 1.0)
    note(f"  {dtype}: max rel {r.max():.2e}  p99 {np.quantile(r, 0.99):.2e}  median {np.median(r):.2e}")
    assert np.array_equal(res.flags.cpu().numpy(), d["ref"].flags)
    assert r.max() < tol
    # detection ranking of the 20 exact-parameter (injection) templates
    order_ref = np.argsort(-ref, kind="stable")
    order = np.argsort(-stat, kind="stable")
    rank_ref = np.empty_like(order_ref)
    rank_ref[order_ref] = np.arange(order_ref.size)
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    inj = np.arange(20)
    note(f"  {dtype}: ranks of the injection templates {np.sort(rank[inj]).tolist()} "
         f"(oracle {np.sort(rank_ref[inj]).tolist()})")
    if dtype == "f32":
        # at FP32 the ranking is the oracle's
        assert np.array_equal(rank[inj], rank_ref[inj])
        assert np.array_equal(order[:200], order_ref[:200])
    else:
        # 16-bit stores: every pair whose oracle values differ by more than twice the store's error bound
        # keeps its order (near-ties at the store's precision may swap)
        lo = ref[inj][:, None] > ref[None, :] * (1.0 + 2.0 * tol) + 2.0 * tol
        hi = ref[inj][:, None] < ref[None, :] * (1.0 - 2.0 * tol) - 2.0 * tol
        si = np.broadcast_to(stat[inj][:, None], lo.shape)
        sj = np.broadcast_to(stat[None, :], lo.shape)
        assert np.all(si[lo] > sj[lo]) and np.all(si[hi] < sj[hi])
