"""A PSD that varies between tranches in a general way (tfsc_transform_tf, the rho factor of tfsc_pixels)
through the C ABI, against the oracle's per-pixel whitening and weights."""
import numpy as np
import pytest
import torch

import tfsc_inputs as ti
from oracle import o2
from oracle import track as otrk
from oracle import transform as otf

from gpu_common import dev, gridspec, lib, note, rel, small_data, tiny_data

pytestmark = pytest.mark.gpu


def _oracle(d, S, x=None):
    g = d["grid"]
    b = d["bank"]
    pix, wt = otf.transform_tf(d["x"] if x is None else x, g, S, d["keep"], 0.1, "rfft")
    res = o2.statistic(pix, None, None, b, g, layout=otrk.Layout(b, g), weight_tf=wt)
    return pix, wt, res


def test_transform_tf_matches_the_oracle():
    """Pixels whitened pixel by pixel (FP64 store, both layer-major layouts) and the weights u_k w_m rho_mk
    against the oracle's keep_m / sqrt(S_m(f_k)); rho is FP32, so the weights agree to FP32 rounding."""
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    S = ti.tranche_psd_tf(g)
    note(f"transform_tf: grid {g.n_bins}x{g.n_tranches}, C={g.n_channels}")
    pix, wt = otf.transform_tf(d["x"], g, S, d["keep"], 0.1, "rfft")
    for layout in ("layer", "layer_ci"):
        st = tfsc.transform_tf(gridspec(g), dev(d["x"]), dev(S), dev(d["keep"]), dtype="f64", layout=layout)
        p = torch.view_as_complex(st.pix).cpu().numpy()
        p = p if layout == "layer" else np.transpose(p, (2, 0, 1))
        scale = np.abs(pix).max()
        assert np.max(np.abs(p - pix)) < 1e-12 * scale, layout
        w = (st.inv_asd.cpu().numpy()[:, None] * st.tranche_w.cpu().numpy()[None, :]
             * st.rho.cpu().numpy().astype(np.float64))
        inner = slice(1, g.n_bins - 1)
        err = np.abs(w[inner] - wt[inner]) / np.abs(wt[inner]).max(axis=None)
        assert err.max() < 2e-7, layout
        assert np.array_equal(st.tranche_w.cpu().numpy() == 0, wt[1] == 0)


@pytest.mark.parametrize("schedule,layout", [("wave", "layer_ci"), ("wave", "layer"), ("thread", "tranche")])
def test_statistic_fp64_against_the_oracle(schedule, layout):
    """FP64 pixels and arithmetic with the drifting-tilt PSD: Upsilon, segment terms and flags."""
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    S = ti.tranche_psd_tf(g)
    note(f"psd_tf statistic f64 {schedule} {layout}")
    _, _, ref = _oracle(d, S)
    st = tfsc.transform_tf(gridspec(g), dev(d["x"]), dev(S), dev(d["keep"]), dtype="f64", layout=layout)
    bt = tfsc.BankTensors.from_host(d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt)
    res = tfsc.bank_statistic(gridspec(g), st, bt, seg, precision="f64", schedule=schedule)
    r = rel(res.stat.cpu().numpy(), ref.stat)
    stt = res.seg_terms[:seg.total].cpu().numpy()
    note(f"  max rel {r.max():.2e}")
    assert r.max() < 1e-6
    assert np.max(np.abs(stt - ref.seg_terms) / np.maximum(ref.seg_terms, 1.0)) < 1e-6
    assert np.array_equal(res.flags.cpu().numpy(), ref.flags)


def test_statistic_fp32_chosen_form_and_ranking():
    """The chosen form (FP32 channel-interleaved store, wave schedule) with the per-pixel PSD: within 1e-4
    of the oracle (given the same FP32-rounded data) and the same best template."""
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    S = ti.tranche_psd_tf(g)
    note("psd_tf statistic f32 wave layer_ci")
    _, _, ref = _oracle(d, S, d["x"].astype(np.float32).astype(np.float64))
    st = tfsc.transform_tf(gridspec(g), dev(d["x"].astype(np.float32)), dev(S), dev(d["keep"]), dtype="f32",
                           layout="layer_ci")
    bt = tfsc.BankTensors.from_host(d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt)
    res = tfsc.bank_statistic(gridspec(g), st, bt, seg, precision="f32", schedule="wave")
    s = res.stat.cpu().numpy()
    r = rel(s, ref.stat)
    note(f"  max rel {r.max():.2e}")
    assert r.max() < 1e-4
    assert int(np.argmax(s)) == int(np.argmax(ref.stat))
    # a different PSD gives a different statistic (the weights are used)
    sep = tfsc.transform(gridspec(g), dev(d["x"].astype(np.float32)), dev(d["psd"]), dev(d["mu"]), dev(d["keep"]),
                         dtype="f32", layout="layer_ci")
    other = tfsc.bank_statistic(gridspec(g), sep, bt, seg, precision="f32", schedule="wave").stat.cpu().numpy()
    assert np.max(np.abs(other - s) / np.maximum(np.abs(s), 1.0)) > 1e-3


@pytest.mark.parametrize("schedule,layout,prec,dtype", [("wave", "layer_ci", "f32", "f32"),
                                                        ("wave", "layer", "f64", "f64"),
                                                        ("wave", "layer_ci", "f64", "f32"),
                                                        ("thread", "tranche", "f32", "f32")])
def test_unit_rho_is_bit_identical_to_the_separable_path(schedule, layout, prec, dtype):
    """rho = 1 multiplies every weight by 1: the same bits as the store without rho."""
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    note(f"unit rho {schedule} {layout} {prec}/{dtype}")
    xx = d["x"] if dtype == "f64" else d["x"].astype(np.float32)
    st = tfsc.transform(gridspec(g), dev(xx), dev(d["psd"]), dev(d["mu"]), dev(d["keep"]), dtype=dtype, layout=layout)
    bt = tfsc.BankTensors.from_host(d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt)
    a = tfsc.bank_statistic(gridspec(g), st, bt, seg, precision=prec, schedule=schedule, want_active=True)
    st1 = tfsc.PixelStore(st.pix, st.inv_asd, st.tranche_w, st.dtype, st.layout, st.layer_scale,
                          torch.ones((g.n_bins, g.n_tranches), dtype=torch.float32, device="cuda"))
    b = tfsc.bank_statistic(gridspec(g), st1, bt, seg, precision=prec, schedule=schedule, want_active=True)
    assert torch.equal(a.stat, b.stat)
    assert torch.equal(a.seg_terms, b.seg_terms)
    assert torch.equal(a.flags, b.flags) and torch.equal(a.n_active, b.n_active)


def test_rho_with_16bit_stores():
    """16-bit stores with rho: refused by the wave schedule, accepted by the thread schedule."""
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    S = ti.tranche_psd_tf(g)
    bt = tfsc.BankTensors.from_host(d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt)
    h = tfsc.transform_tf(gridspec(g), dev(d["x"].astype(np.float32)), dev(S), dev(d["keep"]), dtype="f16",
                          layout="layer_ci")
    with pytest.raises(tfsc.TfscError):  # 16-bit store on the wave schedule
        tfsc.bank_statistic(gridspec(g), h, bt, seg, precision="f32", schedule="wave")
    # the thread schedule takes 16-bit stores with rho: within the F16 store's bar of the oracle
    _, _, ref = _oracle(d, S, d["x"].astype(np.float32).astype(np.float64))
    ht = tfsc.transform_tf(gridspec(g), dev(d["x"].astype(np.float32)), dev(S), dev(d["keep"]), dtype="f16",
                           layout="tranche")
    s = tfsc.bank_statistic(gridspec(g), ht, bt, seg, precision="f32", schedule="thread").stat.cpu().numpy()
    assert rel(s, ref.stat).max() < 2e-3
    assert int(np.argmax(s)) == int(np.argmax(ref.stat))


def test_vjp_with_rho_against_oracle_autograd():
    """The FP64 VJP reads rho like the statistic: against float64 autograd of the oracle with per-pixel weights
    (the same bars as the separable case), and rho = 1 gives the separable VJP bit for bit."""
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    b = d["bank"]
    S = ti.tranche_psd_tf(g)
    lay = otrk.Layout(b, g)
    ok = np.nonzero((lay.flags & (otrk.FLAG_INVALID | otrk.FLAG_EMPTY)) == 0)[0]
    idx = np.concatenate([ok[:5], ok[-3:]])
    note(f"vjp with rho, templates {idx.tolist()}")
    pix, wt = otf.transform_tf(d["x"], g, S, d["keep"], 0.1, "rfft")
    st = tfsc.transform_tf(gridspec(g), dev(d["x"]), dev(S), dev(d["keep"]), dtype="f64", layout="layer_ci")
    bt = tfsc.BankTensors.from_host(b)
    seg = tfsc.segment_layout(gridspec(g), bt)
    fw = tfsc.bank_statistic(gridspec(g), st, bt, seg, precision="f64", want_zn=True)
    ones = torch.ones(bt.n, dtype=torch.float64, device="cuda")
    gp = tfsc.statistic_vjp(gridspec(g), st, bt, seg, fw.seg_zn, g_stat=ones).cpu().numpy()
    ref = np.zeros((len(idx), 5))
    for r, i in enumerate(idx):
        ref[r], _ = o2.gradient(pix, None, None, b, g, int(i), layout=lay, weight_tf=wt)
    floor = 1e-3 * np.max(np.abs(ref), axis=0, keepdims=True)
    err = np.abs(gp[idx] - ref) / np.maximum(np.abs(ref), floor)
    note(f"  max rel vs oracle autograd {err.max():.2e}")
    assert err.max() < 2e-5
    # rho = 1 against no rho, FP32 pixels
    sep = tfsc.transform(gridspec(g), dev(d["x"].astype(np.float32)), dev(d["psd"]), dev(d["mu"]), dev(d["keep"]),
                         dtype="f32", layout="layer_ci")
    one = tfsc.PixelStore(sep.pix, sep.inv_asd, sep.tranche_w, sep.dtype, sep.layout, None,
                          torch.ones((g.n_bins, g.n_tranches), dtype=torch.float32, device="cuda"))
    f1 = tfsc.bank_statistic(gridspec(g), sep, bt, seg, precision="f32", want_zn=True)
    a = tfsc.statistic_vjp(gridspec(g), sep, bt, seg, f1.seg_zn, g_stat=ones)
    c = tfsc.statistic_vjp(gridspec(g), one, bt, seg, f1.seg_zn, g_stat=ones)
    assert torch.equal(a, c)


def test_follow_up_with_a_per_pixel_psd():
    """The Adam follow-up (statistic + VJP + step) on a store whitened by the per-pixel PSD climbs towards the
    tiny injection, as with the separable PSD."""
    tfsc = lib()
    d = tiny_data()
    g = d["grid"]
    inj = ti.TINY_INJECTION
    S = ti.tranche_psd_tf(g)
    note("follow-up with rho on the tiny injection")
    st = tfsc.transform_tf(gridspec(g), dev(d["x"]), dev(S), dev(d["keep"]), dtype="f64", layout="layer_ci")
    rng = np.random.default_rng(11)
    n = 16
    b = ti.Bank(mc=inj["mc"] * np.exp(rng.uniform(-2, 2, n) * 1.4e-3), eta=np.full(n, 0.25),
                f0=inj["f0"] + rng.uniform(-2, 2, n) * 2.5e-7, cos_theta=np.full(n, inj["cos_theta"]) + 0.05,
                phi=np.full(n, inj["phi"]) - 0.05, psi=np.full(n, inj["psi"]),
                cos_iota=np.full(n, inj["cos_iota"]), phase=np.zeros(n))
    bt = tfsc.BankTensors.from_host(b)
    first, best, _ = tfsc.follow_up(gridspec(g), st, bt, steps=30, lr_scale=0.5, nseg_fixed=8, precision="f64")
    first, best = first.cpu().numpy(), best.cpu().numpy()
    one = ti.tiny_bank().subset([256])
    exact = tfsc.bank_statistic(gridspec(g), st, tfsc.BankTensors.from_host(one),
                                tfsc.segment_layout(gridspec(g), tfsc.BankTensors.from_host(one), nseg_fixed=8),
                                precision="f64").stat.item()
    note(f"  exact {exact:.1f}; start median {np.median(first):.1f}; best median {np.median(best):.1f}")
    assert np.all(best >= first)
    assert np.median(best) > 0.9 * exact


def test_several_realisations_with_rho():
    """Three noise realisations whitened by the same per-pixel PSD, in one pass over the bank (groups of 2
    and 1), against one launch per realisation; and rho = 1 against no rho (the rho pass re-sums Q from the
    stored coefficient table, so the two agree to rounding rather than bit for bit)."""
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    S = ti.tranche_psd_tf(g)
    R = 3
    note("several realisations with rho")
    bt = tfsc.BankTensors.from_host(d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt)
    stores = tfsc.realisation_stores(gridspec(g), R, dtype="f32", layout="layer_ci")
    keep = ti.sample_keep_mask(g)[None, :]
    singles = []
    for r in range(R):
        x = (ti.noise(g, realisation=r) * keep).astype(np.float32)
        one = tfsc.transform_tf(gridspec(g), dev(x), dev(S), dev(d["keep"]), dtype="f32", layout="layer_ci")
        stores[r].pix.copy_(one.pix)
        singles.append(one)
    stores[0].inv_asd.copy_(singles[0].inv_asd)
    stores[0].tranche_w.copy_(singles[0].tranche_w)
    stores[0].rho = singles[0].rho
    res = tfsc.bank_statistic_multi(gridspec(g), stores, bt, seg, precision="f32", group=2)
    worst = 0.0
    for r in range(R):
        one = tfsc.bank_statistic(gridspec(g), singles[r], bt, seg, precision="f32", schedule="wave")
        err = rel(res.stat[r].cpu().numpy(), one.stat.cpu().numpy()).max()
        worst = max(worst, err)
        assert err < 2e-6, r
    note(f"  max rel against single launches {worst:.2e}")
    assert not torch.equal(res.stat[0], res.stat[1])
    stores[0].rho = torch.ones_like(singles[0].rho)
    a = tfsc.bank_statistic_multi(gridspec(g), stores, bt, seg, precision="f32", group=2)
    stores[0].rho = None
    b = tfsc.bank_statistic_multi(gridspec(g), stores, bt, seg, precision="f32", group=2)
    assert rel(a.stat.cpu().numpy(), b.stat.cpu().numpy()).max() < 1e-6
