"""LISA response: rigid analytic orbits, single-link responses, TDI A/E.

Paper passages followed (Sec. "Implementation details" and the Outlook):
TDI-2 is approximated by rescaled TDI-1.5 for a rigidly rotating
constellation of constant arm length L ~ 8.3 s with analytic orbits and no
point-ahead; the transfer function is evaluated once per tranche at the
tranche frequency (Eq. (tdi2)) and applied to the whole tranche spectrum.
The single-link transfer functions the paper cites are not printed in it;
the reconstruction used here is the standard one and is stated in full:

* Orbits (first order in the eccentricity e = L / (2 sqrt(3) R), R = 1 AU; or a caller's table of
  positions at the tranche starts, as the Outlook's numerical orbits),
  a = 2 pi t / yr, b_i = 2 pi i / 3 (i = 0, 1, 2):
    p_i = R (cos a, sin a, 0) + (e R / 2) (cos(2a - b_i) - 3 cos b_i,
          sin(2a - b_i) - 3 sin b_i, -2 sqrt(3) cos(a - b_i))       [seconds]
* Source direction (polar theta, azimuth phi); propagation vector
  k = -(sin th cos ph, sin th sin ph, cos th); u = (cos th cos ph,
  cos th sin ph, -sin th), v = (sin ph, -cos ph, 0);
  e+ = cos2psi (uu - vv) + sin2psi (uv + vu),
  ex = -sin2psi (uu - vv) + cos2psi (uv + vu).
* Strain h = A e^{i Phi} carried by the polarisation amplitudes
  a+ = (1 + cos^2 iota) / 2 and ax = -i cos iota.
* Link s -> r (n = unit vector from p_s to p_r, positions at reception time):
    time domain: y_sr(t) = n.[H(t - L - k.p_s) - H(t - k.p_r)].n / (2 (1 - k.n))
    per tranche: G_sr = -i pi f L sinc(pi f L (1 - k.n))
                        exp(-i pi f (L + k.(p_s + p_r))) (a+ n.e+.n + ax n.ex.n)
* TDI-1.5 with equal arms, D = exp(-2 pi i f L):
    X = (1 - D^2)[(y31 + D y13) - (y21 + D y12)], Y, Z cyclic;
    A = (Z - X) / sqrt 2, E = (X - 2Y + Z) / sqrt 6.
  The TDI-2 rescaling is a common factor of A and E and cancels in the
  statistic, so it is omitted.
* Unequal arms (the Outlook's varying arm lengths and point-ahead light
  times): a caller's table of the six link light times L_sr at the tranche
  starts, the geometry frozen over each tranche.  Link s -> r is received
  at p_r after travelling L_sr along the arm direction n_sr, so it left
  from p_r - L_sr n_sr:
    time domain: y_sr(t) = n.[H(t - k.p_r - L_sr (1 - k.n)) - H(t - k.p_r)].n / (2 (1 - k.n))
    per tranche: G_sr = -i pi f L_sr sinc(pi f L_sr (1 - k.n))
                        exp(-i pi f (L_sr (1 - k.n) + 2 k.p_r)) (a+ n.e+.n + ax n.ex.n)
  and first-generation TDI with each path's own delays, D_sr = exp(-2 pi i f L_sr):
    X = (1 - D12 D21)(y31 + D31 y13) - (1 - D13 D31)(y21 + D21 y12), Y, Z cyclic.
  With six equal light times L on a table whose sides are exactly L this is
  the equal-arm form above (p_s = p_r - L n).
* Second-generation TDI on the same frozen geometry (the data the paper
  analyses are TDI-2): with the arms static over the tranche the
  second-generation Michelson combination is the first-generation one
  minus itself delayed by both round trips, X2(t) = X(t) - X(t - R12 - R13)
  (R_ab = L_ab + L_ba), so X2 = (1 - D_R12 D_R13) X; Y, Z cyclic.  For equal
  arms the factor 1 - D^4 is common to X, Y, Z; for unequal arms it differs
  between them and A, E, T are formed from the factored X2, Y2, Z2.
"""
from __future__ import annotations

import math

import torch

PI = 3.141592653589793
CLIGHT = 299792458.0
L_S = 2.5e9 / CLIGHT
AU_S = 1.495978707e11 / CLIGHT
YEAR_S = 31557600.0

# ordered links (sender, receiver), 0-based spacecraft indices
LINKS = [(0, 1), (1, 0), (1, 2), (2, 1), (2, 0), (0, 2)]
# rows of a link light-time table [6][Nt]: each arm's link to the next spacecraft, then the reverse links
LINK_ROWS = [(0, 1), (1, 2), (2, 0), (1, 0), (2, 1), (0, 2)]


def orbits(t):
    """Spacecraft positions [..., 3 spacecraft, 3 coords] in light-seconds."""
    t = t if torch.is_tensor(t) else torch.as_tensor(t, dtype=torch.float64)
    R = AU_S
    e = L_S / (2.0 * math.sqrt(3.0) * R)
    a = 2.0 * PI * t / YEAR_S
    out = []
    for i in range(3):
        b = 2.0 * PI * i / 3.0
        x = R * torch.cos(a) + 0.5 * e * R * (torch.cos(2.0 * a - b) - 3.0 * math.cos(b))
        y = R * torch.sin(a) + 0.5 * e * R * (torch.sin(2.0 * a - b) - 3.0 * math.sin(b))
        z = -math.sqrt(3.0) * e * R * torch.cos(a - b)
        out.append(torch.stack([x, y, z], dim=-1))
    return torch.stack(out, dim=-2)


def sky_frame(cos_theta, phi, psi):
    """(k, e+, ex) for the source direction and polarisation angle."""
    ct = cos_theta if torch.is_tensor(cos_theta) else torch.as_tensor(cos_theta, dtype=torch.float64)
    phi = phi if torch.is_tensor(phi) else torch.as_tensor(phi, dtype=torch.float64)
    psi = psi if torch.is_tensor(psi) else torch.as_tensor(psi, dtype=torch.float64)
    st = torch.sqrt(1.0 - ct * ct)
    cp, sp = torch.cos(phi), torch.sin(phi)
    k = -torch.stack([st * cp, st * sp, ct], dim=-1)
    u = torch.stack([ct * cp, ct * sp, -st], dim=-1)
    v = torch.stack([sp, -cp, torch.zeros_like(cp)], dim=-1)
    uu = u[..., :, None] * u[..., None, :]
    vv = v[..., :, None] * v[..., None, :]
    uv = u[..., :, None] * v[..., None, :]
    ep0 = uu - vv
    ex0 = uv + uv.transpose(-1, -2)
    c2, s2 = torch.cos(2.0 * psi)[..., None, None], torch.sin(2.0 * psi)[..., None, None]
    ep = c2 * ep0 + s2 * ex0
    ex = -s2 * ep0 + c2 * ex0
    return k, ep, ex


def link_lengths(pos):
    """|p_r - p_s| of each link of positions [..., 3, 3] as a table [..., 6] (rows as LINK_ROWS): the light
    times of a constellation whose links have no point-ahead difference."""
    p = torch.as_tensor(pos, dtype=torch.float64)
    return torch.stack([torch.linalg.norm(p[..., r, :] - p[..., s, :], dim=-1) for (s, r) in LINK_ROWS], dim=-1)


def _link_geometry(p, s, r):
    d = p[..., r, :] - p[..., s, :]
    n = d / torch.linalg.norm(d, dim=-1, keepdim=True)
    return n


def _quad(n, e):
    return torch.einsum("...i,...ij,...j->...", n, e, n)


def transfer_ae(t, f, cos_theta, phi, psi, cos_iota):
    """Per-tranche TDI transfer (T_A, T_E) at times t and frequencies f (complex torch).

    cos_theta, phi, psi, cos_iota are 0-d tensors (one template); t and f share
    a shape.
    """
    TA, TE, _ = transfer_aet(t, f, cos_theta, phi, psi, cos_iota)
    return TA, TE


def transfer_aet(t, f, cos_theta, phi, psi, cos_iota, pos=None, links=None, generation: int = 1):
    """(T_A, T_E, T_T): the third channel T = (X + Y + Z) / sqrt 3 completes A and E to an orthonormal
    combination of X, Y, Z (so |T_A|^2 + |T_E|^2 + |T_T|^2 = |T_X|^2 + |T_Y|^2 + |T_Z|^2).  ``pos``: spacecraft
    positions [..., 3, 3] at the times t (a caller's orbit), None for the analytic orbit; ``links``: the six
    link light times [..., 6] at the times t (unequal arms), None for equal arms; ``generation``: TDI 1 or 2
    (2 with a link table)."""
    TX, TY, TZ = transfer_xyz(t, f, cos_theta, phi, psi, cos_iota, pos, links, generation)
    TA = (TZ - TX) / math.sqrt(2.0)
    TE = (TX - 2.0 * TY + TZ) / math.sqrt(6.0)
    TT = (TX + TY + TZ) / math.sqrt(3.0)
    return TA, TE, TT


def transfer_xyz(t, f, cos_theta, phi, psi, cos_iota, pos=None, links=None, generation: int = 1):
    """Per-tranche transfer of the Michelson combinations (T_X, T_Y, T_Z) that A, E and T are formed from.

    ``pos``: spacecraft positions [..., 3 spacecraft, 3 coordinates] (light-seconds) at the times t, for an
    orbit other than the analytic one (Sec. "Outlook": numerical or generic orbits); the arm directions come
    from them, the arm length of the link transfer and the TDI delays stays L.
    ``links``: the six link light times [..., 6] (light-seconds, rows as LINK_ROWS) at the times t; the
    unequal-arm form of the module docstring then replaces the equal-arm one, in the first or (``generation``
    = 2) the second TDI generation."""
    t = t if torch.is_tensor(t) else torch.as_tensor(t, dtype=torch.float64)
    f = f if torch.is_tensor(f) else torch.as_tensor(f, dtype=torch.float64)
    ci = cos_iota if torch.is_tensor(cos_iota) else torch.as_tensor(cos_iota, dtype=torch.float64)
    k, ep, ex = sky_frame(cos_theta, phi, psi)
    p = orbits(t) if pos is None else torch.as_tensor(pos, dtype=torch.float64)
    if links is not None:
        return _transfer_xyz_links(f, k, ep, ex, ci, p, torch.as_tensor(links, dtype=torch.float64), generation)
    if generation != 1:
        raise ValueError("the second TDI generation is formed with a link light-time table")
    ap = (1.0 + ci * ci) / 2.0
    G = {}
    for (s, r) in LINKS:
        n = _link_geometry(p, s, r)
        kn = n @ k
        xp = _quad(n, ep)
        xx = _quad(n, ex)
        amp = torch.complex(ap * xp, -ci * xx)
        x = PI * f * L_S * (1.0 - kn)
        sinc = torch.where(x == 0, torch.ones_like(x), torch.sin(x) / torch.where(x == 0, torch.ones_like(x), x))
        kps = (p[..., s, :] + p[..., r, :]) @ k
        ph = -PI * f * (L_S + kps)
        G[(s, r)] = torch.complex(torch.zeros_like(f), -PI * f * L_S) * sinc * torch.polar(torch.ones_like(ph), ph) * amp
    D = torch.polar(torch.ones_like(f), -2.0 * PI * f * L_S)
    one_m_d2 = 1.0 - D * D
    g = lambda s, r: G[(s - 1, r - 1)]  # 1-based spacecraft labels, sender first
    TX = one_m_d2 * ((g(3, 1) + D * g(1, 3)) - (g(2, 1) + D * g(1, 2)))
    TY = one_m_d2 * ((g(1, 2) + D * g(2, 1)) - (g(3, 2) + D * g(2, 3)))
    TZ = one_m_d2 * ((g(2, 3) + D * g(3, 2)) - (g(1, 3) + D * g(3, 1)))
    return TX, TY, TZ


def _transfer_xyz_links(f, k, ep, ex, ci, p, links, generation=1):
    """(T_X, T_Y, T_Z) with the six link light times ``links`` [..., 6] and positions ``p`` [..., 3, 3]."""
    ap = (1.0 + ci * ci) / 2.0
    G, D = {}, {}
    for row, (s, r) in enumerate(LINK_ROWS):
        L = links[..., row]
        n = _link_geometry(p, s, r)
        kn = n @ k
        amp = torch.complex(ap * _quad(n, ep), -ci * _quad(n, ex))
        x = PI * f * L * (1.0 - kn)
        sinc = torch.where(x == 0, torch.ones_like(x), torch.sin(x) / torch.where(x == 0, torch.ones_like(x), x))
        ph = -PI * f * (L * (1.0 - kn) + 2.0 * (p[..., r, :] @ k))
        G[(s, r)] = torch.complex(torch.zeros_like(f), -PI * f * L) * sinc * torch.polar(torch.ones_like(ph), ph) * amp
        D[(s, r)] = torch.polar(torch.ones_like(f), -2.0 * PI * f * L)
    g = lambda s, r: G[(s - 1, r - 1)]  # 1-based spacecraft labels, sender first
    d = lambda s, r: D[(s - 1, r - 1)]
    TX = (1.0 - d(1, 2) * d(2, 1)) * (g(3, 1) + d(3, 1) * g(1, 3)) - (1.0 - d(1, 3) * d(3, 1)) * (g(2, 1) + d(2, 1) * g(1, 2))
    TY = (1.0 - d(2, 3) * d(3, 2)) * (g(1, 2) + d(1, 2) * g(2, 1)) - (1.0 - d(2, 1) * d(1, 2)) * (g(3, 2) + d(3, 2) * g(2, 3))
    TZ = (1.0 - d(3, 1) * d(1, 3)) * (g(2, 3) + d(2, 3) * g(3, 2)) - (1.0 - d(3, 2) * d(2, 3)) * (g(1, 3) + d(1, 3) * g(3, 1))
    if generation == 2:
        rt = lambda a, b: d(a, b) * d(b, a)  # round trip of the arm between a and b
        TX = (1.0 - rt(1, 2) * rt(1, 3)) * TX
        TY = (1.0 - rt(2, 3) * rt(2, 1)) * TY
        TZ = (1.0 - rt(3, 1) * rt(3, 2)) * TZ
    elif generation != 1:
        raise ValueError("TDI generation 1 or 2")
    return TX, TY, TZ


def tdi_xyz_td_frozen(t, hfun, cos_theta, phi, psi, pos, links, generation: int = 1):
    """Time-domain X, Y, Z at times t for one frozen geometry: positions ``pos`` [3, 3] and the six link light
    times ``links`` [6] (rows as LINK_ROWS), every link and delay of the unequal-arm form written out; the
    second generation as each combination minus itself delayed by its two round trips."""
    k, ep, ex = sky_frame(cos_theta, phi, psi)
    p = torch.as_tensor(pos, dtype=torch.float64)
    Ls = {sr: float(links[row]) for row, sr in enumerate(LINK_ROWS)}

    def y(s, r, tau):
        s0, r0 = s - 1, r - 1
        n = _link_geometry(p, s0, r0)
        kn = float(n @ k)
        kpr = float(p[r0] @ k)
        te = tau - kpr - Ls[(s0, r0)] * (1.0 - kn)
        tr = tau - kpr
        hp_e, hx_e = hfun(te)
        hp_r, hx_r = hfun(tr)
        return ((hp_e - hp_r) * _quad(n, ep) + (hx_e - hx_r) * _quad(n, ex)) / (2.0 * (1.0 - kn))

    def L(s, r):
        return Ls[(s - 1, r - 1)]

    def first(a, b, c, t):
        # centred on a: (1 - R_ab)(y_ca + D_ca y_ac) - (1 - R_ac)(y_ba + D_ba y_ab), R_ab the round trip a -> b -> a
        rab, rac = L(a, b) + L(b, a), L(a, c) + L(c, a)
        return (y(c, a, t) + y(a, c, t - L(c, a)) - y(c, a, t - rab) - y(a, c, t - rab - L(c, a))) \
            - (y(b, a, t) + y(a, b, t - L(b, a)) - y(b, a, t - rac) - y(a, b, t - rac - L(b, a)))

    def michelson(a, b, c, t):
        if generation == 1:
            return first(a, b, c, t)
        return first(a, b, c, t) - first(a, b, c, t - (L(a, b) + L(b, a)) - (L(a, c) + L(c, a)))

    return michelson(1, 2, 3, t), michelson(2, 3, 1, t), michelson(3, 1, 2, t)


def link_td(t, hfun, s, r, k, ep, ex):
    """Time-domain single-link response y_sr(t) for strain callback hfun(t') -> (h+, hx)."""
    p = orbits(t)
    n = _link_geometry(p, s, r)
    kn = n @ k
    xp = _quad(n, ep)
    xx = _quad(n, ex)
    te = t - L_S - p[..., s, :] @ k
    tr = t - p[..., r, :] @ k
    hp_e, hx_e = hfun(te)
    hp_r, hx_r = hfun(tr)
    return ((hp_e - hp_r) * xp + (hx_e - hx_r) * xx) / (2.0 * (1.0 - kn))


def tdi_ae_td(t, hfun, cos_theta, phi, psi):
    """TDI A and E time series at sample times t for strain callback hfun."""
    A, E, _ = tdi_aet_td(t, hfun, cos_theta, phi, psi)
    return A, E


def tdi_aet_td(t, hfun, cos_theta, phi, psi):
    """TDI A, E and T = (X + Y + Z) / sqrt 3 time series at sample times t."""
    k, ep, ex = sky_frame(cos_theta, phi, psi)
    L = L_S

    def y(s, r, delay):
        return link_td(t - delay * L, hfun, s - 1, r - 1, k, ep, ex)

    X = (y(3, 1, 0) + y(1, 3, 1)) - (y(2, 1, 0) + y(1, 2, 1)) \
        - (y(3, 1, 2) + y(1, 3, 3)) + (y(2, 1, 2) + y(1, 2, 3))
    Y = (y(1, 2, 0) + y(2, 1, 1)) - (y(3, 2, 0) + y(2, 3, 1)) \
        - (y(1, 2, 2) + y(2, 1, 3)) + (y(3, 2, 2) + y(2, 3, 3))
    Z = (y(2, 3, 0) + y(3, 2, 1)) - (y(1, 3, 0) + y(3, 1, 1)) \
        - (y(2, 3, 2) + y(3, 2, 3)) + (y(1, 3, 2) + y(3, 1, 3))
    A = (Z - X) / math.sqrt(2.0)
    E = (X - 2.0 * Y + Z) / math.sqrt(6.0)
    T = (X + Y + Z) / math.sqrt(3.0)
    return A, E, T
