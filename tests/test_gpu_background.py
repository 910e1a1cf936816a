"""Per-tile maxima on the device (tfsc_tile_max through the C ABI) and the background over noise realisations."""
import numpy as np
import pytest
import torch

import tfsc_inputs as ti

from gpu_common import dev, gridspec, lib, note, small_data

pytestmark = pytest.mark.gpu


def _numpy_tile_max(stat, tile, n_tiles):
    mx = np.zeros(n_tiles)
    arg = np.full(n_tiles, -1, np.int64)
    for i in range(stat.size):
        t, v = tile[i], stat[i]
        if t < 0 or t >= n_tiles or not v >= 0.0:
            continue
        if arg[t] < 0 or v > mx[t]:
            mx[t], arg[t] = v, i
    return mx, arg


def test_tile_max_matches_numpy_with_ties_exclusions_and_empty_tiles():
    tfsc = lib()
    rng = np.random.default_rng(8)
    n, n_tiles = 200_003, 97
    note(f"tile max: {n} values, {n_tiles} tiles")
    stat = np.round(rng.exponential(30.0, n), 1)  # rounding makes ties within tiles
    stat[rng.integers(0, n, 50)] = np.nan
    stat[rng.integers(0, n, 50)] = -1.0
    stat[rng.integers(0, n, 50)] = -0.0
    tile = rng.integers(-3, n_tiles, n).astype(np.int32)
    tile[tile == 13] = 14  # tile 13 empty
    tile[rng.integers(0, n, 20)] = n_tiles + 5  # out of range: left out
    mx, arg = tfsc.tile_max(dev(stat), dev(tile), n_tiles)
    rmx, rarg = _numpy_tile_max(stat, tile, n_tiles)
    assert np.array_equal(mx.cpu().numpy(), rmx)
    assert np.array_equal(arg.cpu().numpy(), rarg)
    assert arg[13].item() == -1 and mx[13].item() == 0.0
    # empty input: every tile empty
    mx0, arg0 = tfsc.tile_max(dev(np.zeros(0)), dev(np.zeros(0, np.int32)), 5)
    assert torch.all(arg0 == -1) and torch.all(mx0 == 0.0)
    with pytest.raises(tfsc.TfscError):
        tfsc.tile_max(dev(stat), dev(tile), 0)


def test_tile_max_in_a_graph_over_replays():
    tfsc = lib()
    rng = np.random.default_rng(9)
    n, n_tiles = 50_000, 31
    stat = dev(rng.exponential(10.0, n))
    tile = dev(rng.integers(0, n_tiles, n).astype(np.int32))
    out = tfsc.tile_max(stat, tile, n_tiles)
    ref = (out[0].clone(), out[1].clone())
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        tfsc.tile_max(stat, tile, n_tiles, out=out)
    for rep in range(3):
        out[0].fill_(-5.0)
        out[1].fill_(7)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1]), rep
        tfsc.tile_max(stat * 0.5, tile, n_tiles)  # eager work between replays
        torch.cuda.synchronize()


def test_background_over_realisations():
    """Three noise realisations through the realisation graph; per-tile maxima on the device equal the
    maxima of the returned statistic, and the fits run on them."""
    from paper_2510_19047_amd import background as bg
    from paper_2510_19047_amd import batching
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    R = 3
    keep = ti.sample_keep_mask(g)[None, :]
    xs = dev(np.stack([ti.noise(g, realisation=r) * keep for r in range(R)]).astype(np.float32))
    b = d["bank"]
    bt = tfsc.BankTensors.from_host(b)
    seg = tfsc.segment_layout(gridspec(g), bt)
    rg = batching.RealisationGraph(gridspec(g), xs, dev(d["psd"]), dev(d["mu"]), dev(d["keep"]), bt, seg)
    out = rg.replay()
    torch.cuda.synchronize()
    tiles = bg.tile_ids(b.mc, b.f0, np.geomspace(5.0, 100.0, 4), np.linspace(0.004, 0.08, 4))
    B = bg.Background(tiles, 9)
    for r in range(R):
        row = B.add(out[r].stat)
        s = out[r].stat.cpu().numpy()
        ref, _ = _numpy_tile_max(s, tiles, 9)
        assert np.array_equal(row, ref)
    assert B.maxima.shape == (R, 9)
    pl, gb = B.fits()
    note(f"  pooled maxima: Gumbel mu {gb.mu:.1f} beta {gb.beta:.2f}; power-law delta {pl.delta:.2f}")
    assert gb.beta > 0.0 and pl.delta < 0.0
