"""GPU parity of tfsc_transform (window + FFT + whitening + layout + 16-bit stores) against the oracle."""
import numpy as np
import pytest
import torch

from gpu_common import dev, gridspec, lib, note, oracle_stat, rel, small_data, tiny_data

pytestmark = pytest.mark.gpu


def _complex(store):
    p = store.pix.float() if store.pix.dtype in (torch.float16, torch.bfloat16, torch.int16) else store.pix
    z = torch.view_as_complex(p.contiguous().to(torch.float64 if p.dtype == torch.float64 else torch.float32))
    if store.layout == "tranche":
        z = z.transpose(1, 2)
    elif store.layout == "layer_ci":
        z = z.permute(2, 0, 1)
    z = z.to(torch.complex128)
    if store.layer_scale is not None:
        z = z * store.layer_scale.to(torch.float64)[:, :, None]
    return z.cpu().numpy()


def test_tiny_fp64_transform():
    tfsc = lib()
    d = tiny_data()
    g = d["grid"]
    note("transform tiny fp64")
    st = tfsc.transform(gridspec(g, d["alpha"]), dev(d["x"]), dev(d["psd"]), dev(d["mu"]), dev(d["keep"]), dtype="f64")
    z = _complex(st)
    ref = d["pix"]
    err = np.max(np.abs(z - ref)) / np.max(np.abs(ref))
    note(f"  max |diff| / max |D| = {err:.2e}")
    assert err < 1e-12
    assert np.allclose(st.inv_asd.cpu().numpy(), d["u"], rtol=1e-15)
    assert np.array_equal(st.tranche_w.cpu().numpy(), d["wm"])


@pytest.mark.parametrize("layout", ["layer", "tranche", "layer_ci"])
def test_two_channel_fp32_transform(layout):
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    note(f"transform 2ch fp32 {layout}")
    x32 = d["x"].astype(np.float32)
    from oracle import transform as otf
    ref, u, wm = otf.transform(x32.astype(np.float64), g, d["psd"], d["mu"], d["keep"], 0.1, "rfft")
    st = tfsc.transform(gridspec(g), dev(x32), dev(d["psd"]), dev(d["mu"]), dev(d["keep"]), dtype="f32",
                        layout=layout)
    z = _complex(st)
    err = np.max(np.abs(z - ref)) / np.max(np.abs(ref))
    note(f"  max |diff| / max |D| = {err:.2e}")
    assert err < 3e-6
    assert np.array_equal(st.tranche_w.cpu().numpy(), wm)
    assert np.all(z[:, :, d["keep"] == 0] == 0)


@pytest.mark.parametrize("layout", ["layer", "layer_ci"])
@pytest.mark.parametrize("dtype,bits", [("f16", 11), ("bf16", 8)])
def test_16bit_store_with_layer_scale(dtype, bits, layout):
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    note(f"transform {dtype} {layout}")
    x32 = d["x"].astype(np.float32)
    ref32 = tfsc.transform(gridspec(g), dev(x32), dev(d["psd"]), dev(d["mu"]), dev(d["keep"]), dtype="f32")
    st = tfsc.transform(gridspec(g), dev(x32), dev(d["psd"]), dev(d["mu"]), dev(d["keep"]), dtype=dtype,
                        layout=layout)
    z, r = _complex(st), _complex(ref32)
    sc = st.layer_scale.cpu().numpy()
    comp = np.maximum(np.abs(r.real).max(axis=2), np.abs(r.imag).max(axis=2))
    assert np.allclose(sc[comp > 0], comp[comp > 0], rtol=1e-7)
    # every component is within half an ulp of its 16-bit encoding relative to the value
    e = np.maximum(np.abs(z.real - r.real), np.abs(z.imag - r.imag))
    mag = np.maximum(np.abs(r.real), np.abs(r.imag))
    ok = mag > 1e-3 * sc[:, :, None]
    assert np.max(e[ok] / mag[ok]) <= 2.0 ** (-bits) * 1.01


@pytest.mark.parametrize("layout", ["layer", "layer_ci"])
def test_int16_store_on_the_layer_grid(layout):
    """I16 store: layer_scale = layer max / 32767 and every component is the nearest grid point (within half
    a step, plus the FP32 rounding of value x 32767 / max)."""
    tfsc = lib()
    d = small_data()
    g = d["grid"]
    note(f"transform i16 {layout}")
    x32 = d["x"].astype(np.float32)
    ref32 = tfsc.transform(gridspec(g), dev(x32), dev(d["psd"]), dev(d["mu"]), dev(d["keep"]), dtype="f32")
    st = tfsc.transform(gridspec(g), dev(x32), dev(d["psd"]), dev(d["mu"]), dev(d["keep"]), dtype="i16",
                        layout=layout)
    assert st.pix.dtype == torch.int16
    z, r = _complex(st), _complex(ref32)
    sc = st.layer_scale.cpu().numpy().astype(np.float64)
    comp = np.maximum(np.abs(r.real).max(axis=2), np.abs(r.imag).max(axis=2))
    assert np.allclose(sc[comp > 0], comp[comp > 0] / 32767.0, rtol=1e-6)
    q = np.stack([z.real, z.imag]) / np.where(sc > 0, sc, 1.0)[None, :, :, None]
    assert np.max(np.abs(q)) <= 32767.0 + 1e-6 and np.allclose(q, np.rint(q), atol=1e-3)
    e = np.maximum(np.abs(z.real - r.real), np.abs(z.imag - r.imag))
    assert np.all(e <= 0.51 * sc[:, :, None] + 1e-30)


def test_end_to_end_tiny_gpu_transform_then_statistic():
    tfsc = lib()
    d = tiny_data()
    g = d["grid"]
    note("end-to-end tiny: GPU transform -> GPU statistic vs oracle")
    ref = oracle_stat(d)
    st = tfsc.transform(gridspec(g, d["alpha"]), dev(d["x"]), dev(d["psd"]), dev(d["mu"]), dev(d["keep"]), dtype="f64")
    bt = tfsc.BankTensors.from_host(d["bank"])
    seg = tfsc.segment_layout(gridspec(g), bt, nseg_fixed=8)
    res = tfsc.bank_statistic(gridspec(g), st, bt, seg, precision="f64", schedule="wave")
    s = res.stat.cpu().numpy()
    assert rel(s, ref.stat).max() < 1e-6
    assert int(np.argmax(s)) == 256
