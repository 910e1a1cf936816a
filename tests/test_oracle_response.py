"""Pins of the oracle's response model (CPU)."""
import math

import numpy as np
import pytest
import torch

import tfsc_inputs as ti
from oracle import response as rsp
from oracle import track as trk


def test_orbits_rigid_and_tilted():
    t = torch.linspace(0.0, rsp.YEAR_S, 97, dtype=torch.float64)
    p = rsp.orbits(t).numpy()
    for i, j in ((0, 1), (1, 2), (2, 0)):
        arm = np.linalg.norm(p[:, i] - p[:, j], axis=-1)
        assert np.max(np.abs(arm / rsp.L_S - 1)) < 1e-4
    # constellation plane at 60 degrees to the ecliptic, centroid on a 1 AU circle
    nrm = np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
    nrm /= np.linalg.norm(nrm, axis=-1, keepdims=True)
    tilt = np.degrees(np.arccos(np.abs(nrm[:, 2])))
    assert np.max(np.abs(tilt - 60.0)) < 0.05
    cen = p.mean(axis=1)
    assert np.max(np.abs(np.linalg.norm(cen, axis=-1) / rsp.AU_S - 1)) < 1e-4
    # centroid leads by a = 2 pi t / yr
    ang = np.unwrap(np.arctan2(cen[:, 1], cen[:, 0]))
    assert np.allclose(ang, 2 * np.pi * t.numpy() / rsp.YEAR_S, atol=1e-4)


def test_polarisation_tensors():
    k, ep, ex = rsp.sky_frame(torch.tensor(0.37, dtype=torch.float64), torch.tensor(2.1, dtype=torch.float64),
                              torch.tensor(0.8, dtype=torch.float64))
    k, ep, ex = k.numpy(), ep.numpy(), ex.numpy()
    assert abs(np.linalg.norm(k) - 1) < 1e-15
    for e in (ep, ex):
        assert abs(np.trace(e)) < 1e-15
        assert np.allclose(e @ k, 0, atol=1e-15)
        assert np.allclose(e, e.T, atol=0)
        assert abs(np.sum(e * e) - 2) < 1e-14
    assert abs(np.sum(ep * ex)) < 1e-15
    # source direction opposite to propagation: (theta, phi) -> -(sin th cos ph, ...)
    st = math.sqrt(1 - 0.37 ** 2)
    assert np.allclose(-k, [st * math.cos(2.1), st * math.sin(2.1), 0.37], atol=1e-15)


def _xi(n, ep, ex, ci):
    ap = (1 + ci * ci) / 2
    return ap * (n @ ep @ n) - 1j * ci * (n @ ex @ n)


def test_long_wavelength_limit_of_tdi_x():
    """For f L -> 0 the first-generation Michelson X reduces to 8 (pi f L)^2 (xi_13 - xi_12)
    (xi = n.(a+ e+ + ax ex).n of each arm), up to the common propagation phase."""
    ct, ph, ps, ci = 0.2, 1.3, 0.5, 0.4
    t = torch.tensor([1.0e6], dtype=torch.float64)
    f = torch.tensor([1e-8], dtype=torch.float64)
    TA, TE = rsp.transfer_ae(t, f, ct, ph, ps, ci)
    k, ep, ex = (a.numpy() for a in rsp.sky_frame(torch.tensor(ct, dtype=torch.float64),
                                                  torch.tensor(ph, dtype=torch.float64),
                                                  torch.tensor(ps, dtype=torch.float64)))
    p = rsp.orbits(t).numpy()[0]

    def unit(a, b):
        d = p[b] - p[a]
        return d / np.linalg.norm(d)

    xi = {}
    for (s, r) in ((0, 1), (0, 2), (1, 2)):
        xi[(s, r)] = _xi(unit(s, r), ep, ex, ci)
    # plus the propagation phase from the solar-system barycentre to the constellation
    pref = 8 * (math.pi * float(f[0]) * rsp.L_S) ** 2 * np.exp(-2j * math.pi * float(f[0]) * (k @ p.mean(axis=0)))
    X = pref * (xi[(0, 2)] - xi[(0, 1)])
    Y = pref * (xi[(0, 1)] - xi[(1, 2)])
    Z = pref * (xi[(1, 2)] - xi[(0, 2)])
    A = (Z - X) / math.sqrt(2)
    E = (X - 2 * Y + Z) / math.sqrt(6)
    assert abs(complex(TA[0]) / A - 1) < 1e-4
    assert abs(complex(TE[0]) / E - 1) < 1e-4


@pytest.mark.parametrize("ct,ph,ps,ci", [(0.3, 1.0, 0.4, 0.6), (-0.8, 4.0, 2.2, -0.1)])
def test_time_domain_response_matches_transfer(ct, ph, ps, ci):
    """TD single links + TDI with explicit delays vs T(t, f) A e^{i Phi} (the two forms of the response)."""
    tpl = trk.Template(torch.tensor(30.0, dtype=torch.float64), torch.tensor(0.25, dtype=torch.float64),
                       torch.tensor(0.02, dtype=torch.float64))
    ap = (1 + ci * ci) / 2

    def hfun(tq):
        Phi, f, fdot, A = tpl.at(tq)
        e = torch.polar(torch.ones_like(Phi), Phi)
        return A * ap * e, A * torch.complex(torch.zeros_like(Phi), -ci * torch.ones_like(Phi)) * e

    t = torch.linspace(1e5, 3e7, 50, dtype=torch.float64)
    A_td, E_td = rsp.tdi_ae_td(t, hfun, ct, ph, ps)
    Phi, f, _, Am = tpl.at(t)
    TA, TE = rsp.transfer_ae(t, f, ct, ph, ps, ci)
    carrier = Am * torch.polar(torch.ones_like(Phi), Phi)
    for td, T in ((A_td, TA), (E_td, TE)):
        ref = T * carrier
        err = (td - ref).abs() / ref.abs().max()
        assert float(err.max()) < 2e-3
