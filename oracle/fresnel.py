"""Fresnel integrals and the Fresnel-kernel tranche spectrum.

Paper passages followed:
* Eq. (fresnel-ft): over one tranche the spectrum of A e^{i phi(t)} with a
  quadratic phase is A / sqrt(2 fdot) exp(i(phi_nm - pi fdot zeta^2)) F(f),
  zeta = (f_nm - f) / fdot.
* Eq. (kernel-function): F = Delta C + i Delta S, with the Fresnel integrals
  taken between v(t_nm) and v(t_{n m+1}), v = sqrt(2 fdot) [(t - t_nm) + zeta].
* Fresnel approximations: for |z| > 6 the one-term asymptotic forms; for
  |z| <= 6 the rational forms with the f(z), g(z) coefficients the paper
  prints; S and C are odd in z.

Readings: |z| = 6 exactly takes the rational branch; the rational forms are
evaluated at |z| and the sign is applied afterwards (so S(0) = C(0) = 0);
the tranche time origin is the tranche start (the paper's v carries no
e^{-2 pi i f t_nm} factor).
"""
from __future__ import annotations

import numpy as np
import torch

from .track import crsqrt

PI = 3.141592653589793


def fresnel_paper(z):
    """(C(z), S(z)) by the paper's two-branch approximation (torch float64)."""
    z = z if torch.is_tensor(z) else torch.as_tensor(z, dtype=torch.float64)
    az = torch.abs(z)
    sgn = torch.sign(z)
    arg = (PI / 2.0) * az * az
    c, s = torch.cos(arg), torch.sin(arg)
    big = az > 6.0
    # asymptotic branch (|z| > 6); keep the unused lanes finite for autograd
    az_a = torch.where(big, az, torch.full_like(az, 7.0))
    S_a = 0.5 - c / (PI * az_a)
    C_a = 0.5 + s / (PI * az_a)
    # rational branch (|z| <= 6)
    az_r = torch.where(big, torch.zeros_like(az), az)
    fz = (1.0 + 0.926 * az_r) / (2.0 + 1.792 * az_r + 3.104 * az_r * az_r)
    gz = 1.0 / (2.0 + 4.142 * az_r + 3.492 * az_r * az_r + 6.670 * az_r * az_r * az_r)
    S_r = 0.5 - fz * c - gz * s
    C_r = 0.5 + fz * s - gz * c
    C = torch.where(big, C_a, C_r) * sgn
    S = torch.where(big, S_a, S_r) * sgn
    return C, S


def fresnel_exact(z):
    """(C(z), S(z)) from scipy (library reference; numpy in, numpy out)."""
    from scipy.special import fresnel
    S, C = fresnel(np.asarray(z, dtype=np.float64))
    return C, S


def tranche_spectrum(Phi, f, fdot, A, fk, dT, exact: bool = False):
    """Eq. (fresnel-ft): the tranche spectrum h~(f_k), complex torch tensor.

    Phi, f, fdot, A broadcast against the bin frequencies fk (Hz); dT is the
    tranche length.  ``exact`` swaps the paper's Fresnel approximation for
    scipy's Fresnel integrals (no autograd in that mode).
    """
    Phi, f, fdot, A, fk = (x if torch.is_tensor(x) and x.dtype == torch.float64
                           else torch.as_tensor(x, dtype=torch.float64) for x in (Phi, f, fdot, A, fk))
    zeta = (f - fk) / fdot
    r = crsqrt(2.0 * fdot)
    v0 = r * zeta
    v1 = r * (dT + zeta)
    if exact:
        C1, S1 = (torch.as_tensor(a) for a in fresnel_exact(v1.detach().numpy()))
        C0, S0 = (torch.as_tensor(a) for a in fresnel_exact(v0.detach().numpy()))
    else:
        C1, S1 = fresnel_paper(v1)
        C0, S0 = fresnel_paper(v0)
    dC = C1 - C0
    dS = S1 - S0
    ph = Phi - PI * fdot * zeta * zeta
    pref = A / r
    re = pref * (torch.cos(ph) * dC - torch.sin(ph) * dS)
    im = pref * (torch.sin(ph) * dC + torch.cos(ph) * dS)
    return torch.complex(re, im)
