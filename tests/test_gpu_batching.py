"""Batching: HIP-graph replay over noise realisations and launch-shape autotuning (through the C ABI)."""
import json

import numpy as np
import pytest
import torch

import tfsc_inputs as ti

from gpu_common import dev, gridspec, lib, note, oracle_stat, small_data

pytestmark = pytest.mark.gpu


def _realisations(g, R):
    keep = ti.sample_keep_mask(g)[None, :]
    return np.stack([ti.noise(g, realisation=r) * keep for r in range(R)]).astype(np.float32)


def test_graph_replay_matches_eager_over_realisations():
    from paper_2510_19047_amd import batching
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    R = 3
    note(f"graph over {R} realisations")
    xs = dev(_realisations(g, R))
    bt = tfsc.BankTensors.from_host(d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt)
    order = tfsc.processing_order(gridspec(g), bt)
    rg = batching.RealisationGraph(gridspec(g), xs, dev(d["psd"]), dev(d["mu"]), dev(d["keep"]), bt, seg,
                                   store="f32", precision="f32", order=order)
    eager = [r.stat.clone() for r in rg.eager()]
    torch.cuda.synchronize()
    # each realisation on its own, through the plain calls
    for r in range(R):
        st = tfsc.transform(gridspec(g), xs[r], dev(d["psd"]), dev(d["mu"]), dev(d["keep"]), dtype="f32")
        one = tfsc.bank_statistic(gridspec(g), st, bt, seg, precision="f32", schedule="wave")
        assert torch.equal(one.stat, eager[r])
    assert not torch.equal(eager[0], eager[1])
    for rep in range(3):
        for res in rg.results:
            res.stat.fill_(-1.0)
        out = rg.replay()
        torch.cuda.synchronize()
        for r in range(R):
            assert torch.equal(out[r].stat, eager[r]), (rep, r)
        # eager work between replays
        tfsc.bank_statistic(gridspec(g), rg.stores[0], bt, seg, precision="f32", schedule="wave")
        torch.cuda.synchronize()
    note("  3 replays equal the eager results")


def test_realisation_zero_against_oracle():
    """The first realisation of the graph equals the FP64 oracle to the FP32 bar."""
    from paper_2510_19047_amd import batching
    from oracle import transform as otf
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    xs = _realisations(g, 1)
    rg = batching.RealisationGraph(gridspec(g), dev(xs), dev(d["psd"]), dev(d["mu"]), dev(d["keep"]),
                                   tfsc.BankTensors.from_host(d["bank"]),
                                   tfsc.segment_layout(gridspec(g), tfsc.BankTensors.from_host(d["bank"])))
    out = rg.replay()
    torch.cuda.synchronize()
    pix, u, wm = otf.transform(xs[0].astype(np.float64), g, d["psd"], d["mu"], d["keep"], 0.1, "rfft")
    ref = oracle_stat(dict(d, pix=pix, u=u, wm=wm))
    s = out[0].stat.cpu().numpy()
    assert np.max(np.abs(s - ref.stat) / np.maximum(np.abs(ref.stat), 1.0)) < 1e-4


def test_autotune_picks_a_candidate_and_caches(tmp_path):
    from paper_2510_19047_amd import batching
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    note("autotune")
    bt = tfsc.BankTensors.from_host(ti.random_bank(2048, 7, mc_range=(5.0, 100.0), f0_range=(0.004, 0.08),
                                                   stream=9))
    seg = tfsc.segment_layout(gridspec(g), bt)
    store = tfsc.transform(gridspec(g), dev(d["x"].astype(np.float32)), dev(d["psd"]), dev(d["mu"]),
                           dev(d["keep"]), dtype="f32")
    path = str(tmp_path / "shapes.json")
    shape = batching.autotune(gridspec(g), store, bt, seg, cache=path)
    assert shape in ((4, 4), (4, 3), (4, 2), (2, 8), (2, 6), (2, 4), (1, 12), (1, 8))
    with open(path) as fh:
        table = json.load(fh)
    assert len(table) == 1 and tuple(next(iter(table.values()))["shape"]) == shape
    # cached: no re-timing, same answer
    assert batching.autotune(gridspec(g), store, bt, seg, cache=path) == shape
    # the library keeps the tuned shape under its key: a launch with that tune key uses it, and gives the same
    # results as the explicit shape
    key = next(iter(table))
    a = tfsc.bank_statistic(gridspec(g), store, bt, seg, precision="f32", schedule="wave", tune_key=key)
    b = tfsc.bank_statistic(gridspec(g), store, bt, seg, precision="f32", schedule="wave", block_waves=shape[0],
                            groups_per_cu=shape[1])
    assert torch.equal(a.stat, b.stat)


def test_multi_graph_replay_matches_eager_and_single_launches():
    """The several-realisation graph: replays equal the eager multi launch bit for bit, and each realisation
    agrees with its own single-realisation launch to FP32 rounding."""
    from paper_2510_19047_amd import batching
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    R = 3
    note(f"multi-realisation graph over {R} realisations")
    xs = dev(_realisations(g, R))
    bt = tfsc.BankTensors.from_host(d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt)
    rg = batching.RealisationGraph(gridspec(g), xs, dev(d["psd"]), dev(d["mu"]), dev(d["keep"]), bt, seg,
                                   store="f32", precision="f32", multi=True)
    eager = [r.stat.clone() for r in rg.eager()]
    torch.cuda.synchronize()
    for r in range(R):
        one = tfsc.bank_statistic(gridspec(g), rg.stores[r], bt, seg, precision="f32", schedule="wave")
        a, b = eager[r].cpu().numpy(), one.stat.cpu().numpy()
        assert np.max(np.abs(a - b) / np.maximum(np.abs(b), 1.0)) < 2e-6
    for rep in range(3):
        rg.multi_result.stat.fill_(-1.0)
        out = rg.replay()
        torch.cuda.synchronize()
        for r in range(R):
            assert torch.equal(out[r].stat, eager[r]), (rep, r)
        tfsc.bank_statistic(gridspec(g), rg.stores[0], bt, seg, precision="f32", schedule="wave")
        torch.cuda.synchronize()
