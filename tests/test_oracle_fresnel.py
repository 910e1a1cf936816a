"""Pins of the oracle's Fresnel forms and tranche spectrum (CPU)."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import fresnel

HERE = os.path.dirname(os.path.abspath(__file__))


def test_paper_forms_against_scipy():
    # rational branch |z| <= 6 and asymptotic branch |z| > 6, measured against scipy
    z = np.concatenate([np.linspace(0, 6, 6001), np.linspace(6.0001, 60, 20000)])
    C, S = fresnel.fresnel_paper(torch.tensor(z))
    Ce, Se = fresnel.fresnel_exact(z)
    err = np.maximum(np.abs(C.numpy() - Ce), np.abs(S.numpy() - Se))
    rat = z <= 6
    # the printed coefficients reach ~2.2e-3 (rational) and ~4.7e-4 (asymptotic at |z| = 6),
    # not the 1e-4 the text claims; a wrong digit in any coefficient exceeds these bounds
    assert err[rat].max() < 2.5e-3
    assert err[~rat].max() < 5.0e-4
    assert err[z > 20].max() < 1e-4


def test_odd_and_zero():
    z = torch.tensor([-7.5, -3.2, -0.4, 0.0, 0.4, 3.2, 7.5], dtype=torch.float64)
    C, S = fresnel.fresnel_paper(z)
    assert torch.allclose(C, -C.flip(0), atol=0) and torch.allclose(S, -S.flip(0), atol=0)
    assert float(C[3]) == 0.0 and float(S[3]) == 0.0


def test_golden_printed_coefficients():
    with open(os.path.join(HERE, "golden", "paper_constants.json")) as fh:
        gold = json.load(fh)
    fn = gold["fresnel_rational_f"]["value"]
    gn = gold["fresnel_rational_g"]["value"]
    z = np.array([0.3, 1.7, 4.9])
    f = (fn["num"][0] + fn["num"][1] * z) / (fn["den"][0] + fn["den"][1] * z + fn["den"][2] * z * z)
    g = 1.0 / (gn["den"][0] + gn["den"][1] * z + gn["den"][2] * z ** 2 + gn["den"][3] * z ** 3)
    arg = np.pi * z * z / 2
    S_gold = 0.5 - f * np.cos(arg) - g * np.sin(arg)
    C_gold = 0.5 + f * np.sin(arg) - g * np.cos(arg)
    C, S = fresnel.fresnel_paper(torch.tensor(z))
    assert np.allclose(C.numpy(), C_gold, rtol=0, atol=1e-15)
    assert np.allclose(S.numpy(), S_gold, rtol=0, atol=1e-15)
    zs = gold["fresnel_switch"]["value"]
    za = np.array([zs + 0.5, 2 * zs])
    Ca, Sa = fresnel.fresnel_paper(torch.tensor(za))
    assert np.allclose(Sa.numpy(), 0.5 - np.cos(np.pi * za ** 2 / 2) / (np.pi * za), atol=1e-15)
    assert np.allclose(Ca.numpy(), 0.5 + np.sin(np.pi * za ** 2 / 2) / (np.pi * za), atol=1e-15)


def _quadrature_chirp_ft(Phi, f, fdot, A, fk, dT, n=20001):
    """Reference: integral over one tranche of A exp(i(Phi + 2 pi f s + pi fdot s^2 - 2 pi fk s)) ds
    by composite Simpson's rule on a fine grid (independent of the Fresnel closed form)."""
    s = np.linspace(0.0, dT, n)
    ph = Phi + 2 * np.pi * (f - fk[:, None]) * s[None, :] + np.pi * fdot * s[None, :] ** 2
    y = A * np.exp(1j * ph)
    from scipy.integrate import simpson
    return simpson(y, x=s, axis=1)


@pytest.mark.parametrize("fdot", [3e-11, 4e-9, 2.5e-7])
def test_tranche_spectrum_exact_fresnel_matches_quadrature(fdot):
    dT = 2560.0
    f = 0.0150123
    Phi, A = 1.234, 2.0
    kc = np.ceil(f * dT)
    fk = (kc + np.arange(-10, 11)) / dT
    h = fresnel.tranche_spectrum(Phi, f, fdot, A, fk, dT, exact=True).numpy()
    ref = _quadrature_chirp_ft(Phi, f, fdot, A, fk, dT)
    assert np.max(np.abs(h - ref)) / np.max(np.abs(ref)) < 1e-9


@pytest.mark.parametrize("fdot", [3e-11, 4e-9, 2.5e-7])
def test_tranche_spectrum_paper_forms_close(fdot):
    dT = 2560.0
    f = 0.0150123
    kc = np.ceil(f * dT)
    fk = (kc + np.arange(-10, 11)) / dT
    args = (0.3, f, fdot, 1.0, fk, dT)
    hp = fresnel.tranche_spectrum(*args).numpy()
    he = fresnel.tranche_spectrum(*args, exact=True).numpy()
    match = np.abs(np.vdot(hp, he)) / np.sqrt(np.vdot(hp, hp).real * np.vdot(he, he).real)
    assert match > 0.9999
    # per bin the error is at most the Fresnel error (2.5e-3 per integral, two integrals, C and S)
    # times the prefactor A / sqrt(2 fdot)
    bound = 4 * 2.5e-3 / np.sqrt(2 * fdot)
    assert np.max(np.abs(hp - he)) < bound
