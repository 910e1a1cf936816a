"""Seeded synthetic inputs for the semi-coherent time-frequency search.

This module is the only code that both the FP64 oracle and the HIP path's
tests use.  It draws random numbers and writes out the *inputs* of the
statistic (noise time series, the noise PSD model, gap and modulation masks,
template-bank and injection parameters).  It holds none of the statistic's
own arithmetic: no track, no response, no transform, no Fresnel kernel.

Workloads (shapes follow the paper's data set: two years of TDI A/E at a
5 s cadence, hour-scale tranches, sources in the 5-100 Msun / 1-100 mHz
range, gaps; paper Sec. "Searching the Yorsh dataset" and "Search extension
to data with gaps").  The LDC data set and its PSD are not available; these
synthetic stand-ins replace them:

* ``tiny``   0.1 yr, channel A only, dt = 5 s, M = 512, Nt = 1232.
* ``full``   2 yr, channels A and E, dt = 5 s, M = 2048, Nt = 6144,
             +-20 % PSD modulation on a 1-yr sinusoid, 7-h gaps every 14 d.

All randomness comes from PCG64 generators seeded with
``SeedSequence([20251019, cfg_id, stream_id])``; stream ids are
0 noise, 1 injections, 2 bank, 3 gap/PSD phases, 100 + r noise realisation r.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_ROOT = 20251019
STREAM_NOISE = 0
STREAM_INJ = 1
STREAM_BANK = 2
STREAM_GAPS = 3
STREAM_REAL0 = 100

CLIGHT = 299792458.0
L_ARM_M = 2.5e9
YEAR_S = 31557600.0
DAY_S = 86400.0


def rng(cfg_id: int, stream_id: int) -> np.random.Generator:
    """Counter-free PCG64 generator for (config, stream)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, cfg_id, stream_id])))


@dataclass(frozen=True)
class GridSpec:
    """Sampling grid: C channels of N = Nt * M samples at cadence dt."""
    name: str
    cfg_id: int
    n_channels: int
    dt: float
    tranche_len: int           # M samples per tranche
    n_tranches: int            # Nt
    modulated: bool = False    # +-20 % PSD modulation on a 1-yr sinusoid
    gapped: bool = False       # 7-h gaps every 14 d, first at day 7
    nseg_fixed: int = 0        # 0 = per-template rule from fdot0

    @property
    def n_samples(self) -> int:
        return self.tranche_len * self.n_tranches

    @property
    def tranche_dur(self) -> float:
        return self.tranche_len * self.dt

    @property
    def n_bins(self) -> int:
        return self.tranche_len // 2 + 1


TINY = GridSpec("tiny", 1, 1, 5.0, 512, 1232, nseg_fixed=8)
FULL = GridSpec("full", 2, 2, 5.0, 2048, 6144, modulated=True, gapped=True)


def custom_grid(n_channels: int, tranche_len: int, n_tranches: int, dt: float = 5.0,
                modulated: bool = False, gapped: bool = False, nseg_fixed: int = 0,
                cfg_id: int = 9) -> GridSpec:
    return GridSpec(f"custom{n_channels}x{tranche_len}x{n_tranches}", cfg_id, n_channels, dt,
                    tranche_len, n_tranches, modulated, gapped, nseg_fixed)


# ---------------------------------------------------------------- noise model
def lisa_like_psd_ae(f):
    """Analytic one-sided PSD of TDI A (= E) in fractional-frequency units.

    Stand-in for the LDC "Sangria" model (which is not available):
    equal-arm TDI-1.5 A/E noise from an acceleration term and an
    optical-metrology term, arm length 2.5e9 m.
    """
    f = np.asarray(f, dtype=np.float64)
    L = L_ARM_M / CLIGHT
    w = 2.0 * np.pi * f
    s_acc = (3e-15) ** 2 * (1.0 + (4e-4 / f) ** 2) * (1.0 + (f / 8e-3) ** 4) / (w * CLIGHT) ** 2
    s_oms = (15e-12) ** 2 * (1.0 + (2e-3 / f) ** 4) * (w / CLIGHT) ** 2
    c1 = np.cos(w * L)
    c2 = np.cos(2.0 * w * L)
    return 8.0 * np.sin(w * L) ** 2 * ((2.0 + c1) * s_oms + 2.0 * (3.0 + 2.0 * c1 + c2) * s_acc)


def psd_on_bins(grid: GridSpec, alpha: float = 0.1, reach: int = 32, oversample: int = 16) -> np.ndarray:
    """Whitening PSD S0_k at the tranche bins f_k = k / (M dt), k = 0..M/2 (bin 0 copies bin 1).

    S0_k is the analytic PSD averaged over the spectral window of one tranche (Tukey(alpha), M
    samples): S0_k = sum_nu S(f_k + nu) K(nu) / sum_nu K(nu), K = |W(nu)|^2 on a grid of step
    1/(oversample M dt) over +-reach bins.  This is the expected periodogram of the noise at bin k,
    so the whitened pixels have unit variance also at the TDI null f = 1/(2L), whose width is far
    below one bin (there the PSD at the bin centre is 1e3 times below the tranche's average power).
    Frequencies below 0 and above Nyquist are folded back; the lowest bins (far below the band of
    any template here) see only the window's main lobe and near sidelobes.
    """
    M, dT = grid.tranche_len, grid.tranche_dur
    if alpha <= 0.0:
        w = np.ones(M)
    else:
        from scipy.signal.windows import tukey
        w = tukey(M, alpha)
    n_fine = oversample * M
    K = np.abs(np.fft.fft(w, n=n_fine)) ** 2
    q = np.arange(-reach * oversample, reach * oversample + 1)
    Kq = K[q % n_fine]
    Kq = Kq / Kq.sum()
    nu = q / (oversample * dT)
    fnyq = 0.5 / grid.dt
    k = np.arange(grid.n_bins, dtype=np.float64)
    f = k[:, None] / dT + nu[None, :]
    f = np.abs(f)
    f = np.where(f > fnyq, 2.0 * fnyq - f, f)
    f = np.maximum(f, 1.0 / (oversample * dT))
    out = (lisa_like_psd_ae(f) * Kq[None, :]).sum(axis=1)
    out[0] = out[1]
    return out


def modulation(t) -> np.ndarray:
    """PSD multiplier mu(t) = 1 + 0.2 sin(2 pi t / yr)."""
    return 1.0 + 0.2 * np.sin(2.0 * np.pi * np.asarray(t, dtype=np.float64) / YEAR_S)


def tranche_psd_scale(grid: GridSpec) -> np.ndarray:
    """mu_m evaluated at the middle of each tranche (1 for unmodulated grids)."""
    if not grid.modulated:
        return np.ones(grid.n_tranches)
    tm = (np.arange(grid.n_tranches) + 0.5) * grid.tranche_dur
    return modulation(tm)


def tranche_psd_tf(grid: GridSpec, tilt: float = 0.3, period_s: float = 0.5 * YEAR_S) -> np.ndarray:
    """A locally stationary PSD that is not separable in time and frequency, S[K, Nt] = S_m(f_k):
    mu_m S0_k times a spectral tilt that drifts with time, (f_k / 10 mHz)^(gamma_m) with
    gamma_m = tilt sin(2 pi t_m / period + 0.7) at the middle of each tranche (bin 0 uses bin 1's
    frequency).  Like a confusion-noise foreground whose shape changes over the orbit."""
    S0 = psd_on_bins(grid)
    mu = tranche_psd_scale(grid)
    tm = (np.arange(grid.n_tranches) + 0.5) * grid.tranche_dur
    gamma = tilt * np.sin(2.0 * np.pi * tm / period_s + 0.7)
    fk = np.maximum(np.arange(grid.n_bins, dtype=np.float64), 1.0) / grid.tranche_dur
    return S0[:, None] * mu[None, :] * np.power(fk[:, None] / 0.01, gamma[None, :])


def gap_intervals(grid: GridSpec):
    """List of (start, stop) seconds of the scheduled 7-h gaps (every 14 d from day 7)."""
    if not grid.gapped:
        return []
    T = grid.n_samples * grid.dt
    out = []
    g = 0
    while True:
        s = (7.0 + 14.0 * g) * DAY_S
        if s >= T:
            break
        out.append((s, min(s + 7.0 * 3600.0, T)))
        g += 1
    return out


def sample_keep_mask(grid: GridSpec) -> np.ndarray:
    """1.0 outside gaps, 0.0 inside (length N)."""
    keep = np.ones(grid.n_samples)
    t = np.arange(grid.n_samples) * grid.dt
    for s, e in gap_intervals(grid):
        keep[(t >= s) & (t < e)] = 0.0
    return keep


def tranche_keep(grid: GridSpec) -> np.ndarray:
    """uint8 per tranche: 0 if the tranche [m dT, (m+1) dT) overlaps a gap."""
    keep = np.ones(grid.n_tranches, dtype=np.uint8)
    dT = grid.tranche_dur
    for s, e in gap_intervals(grid):
        m0 = int(math.floor(s / dT))
        m1 = int(math.ceil(e / dT))
        keep[m0:min(m1, grid.n_tranches)] = 0
    return keep


def noise(grid: GridSpec, realisation: int | None = None, dtype=np.float64) -> np.ndarray:
    """Stationary Gaussian noise coloured by the A/E PSD, [C][N].

    Drawn in the frequency domain: X_k = sqrt(N S(f_k) / (4 dt)) (a + i b),
    a, b ~ N(0, 1), X_0 = X_{N/2} = 0, x = irfft(X).  For modulated grids the
    series is multiplied by sqrt(mu(t)).  Gaps are NOT applied here (the
    caller zeroes gap samples after adding signals).
    """
    stream = STREAM_NOISE if realisation is None else STREAM_REAL0 + realisation
    g = rng(grid.cfg_id, stream)
    N = grid.n_samples
    nf = N // 2 + 1
    f = np.arange(nf, dtype=np.float64) / (N * grid.dt)
    S = np.zeros(nf)
    S[1:-1] = lisa_like_psd_ae(f[1:-1])
    amp = np.sqrt(N * S / (4.0 * grid.dt))
    out = np.empty((grid.n_channels, N), dtype=dtype)
    sqmu = np.sqrt(modulation(np.arange(N) * grid.dt)) if grid.modulated else None
    for c in range(grid.n_channels):
        X = amp * (g.standard_normal(nf) + 1j * g.standard_normal(nf))
        x = np.fft.irfft(X, n=N)
        if sqmu is not None:
            x *= sqmu
        out[c] = x
    return out


def white_noise(grid: GridSpec, seed_stream: int = 7, sigma: float = 1.0) -> np.ndarray:
    """Unit white Gaussian noise [C][N] (for noise-law checks)."""
    g = rng(grid.cfg_id, seed_stream)
    return sigma * g.standard_normal((grid.n_channels, grid.n_samples))


def pixel_noise(shape, cfg_id: int = 9, stream: int = 11) -> np.ndarray:
    """i.i.d. circular complex normal pixels CN(0, 1): E|z|^2 = 1."""
    g = rng(cfg_id, stream)
    return (g.standard_normal(shape) + 1j * g.standard_normal(shape)) / math.sqrt(2.0)


# ---------------------------------------------------------------- parameters
@dataclass
class Bank:
    """Structure-of-arrays template parameters (FP64).

    mc [Msun] chirp mass, eta symmetric mass ratio, f0 [Hz] GW frequency at
    t = 0, cos_theta / phi sky direction (polar / azimuth, ecliptic frame),
    psi polarisation angle, cos_iota inclination.
    """
    mc: np.ndarray
    eta: np.ndarray
    f0: np.ndarray
    cos_theta: np.ndarray
    phi: np.ndarray
    psi: np.ndarray
    cos_iota: np.ndarray
    phase: np.ndarray = field(default=None)  # injections only: constant phase offset

    FIELDS = ("mc", "eta", "f0", "cos_theta", "phi", "psi", "cos_iota")

    def __len__(self):
        return len(self.mc)

    def subset(self, idx) -> "Bank":
        idx = np.asarray(idx)
        kw = {k: np.ascontiguousarray(getattr(self, k)[idx]) for k in self.FIELDS}
        kw["phase"] = None if self.phase is None else np.ascontiguousarray(self.phase[idx])
        return Bank(**kw)

    @staticmethod
    def concat(a: "Bank", b: "Bank") -> "Bank":
        kw = {k: np.concatenate([getattr(a, k), getattr(b, k)]) for k in Bank.FIELDS}
        return Bank(**kw)

    def as_dict(self):
        return {k: getattr(self, k) for k in self.FIELDS}


def _q_to_eta(q):
    return q / (1.0 + q) ** 2


TINY_INJECTION = dict(mc=30.0, eta=0.25, f0=0.015, cos_theta=0.3, phi=1.0, psi=0.4, cos_iota=0.6,
                      phase=0.7, snr=20.0)


def tiny_injection() -> Bank:
    p = TINY_INJECTION
    return Bank(*(np.array([p[k]]) for k in Bank.FIELDS), phase=np.array([p["phase"]]))


def tiny_bank() -> Bank:
    """16 x 16 grid in (ln Mc in [ln 20, ln 40], f0 in [14, 16] mHz) at the
    injection's sky / polarisation / inclination, plus one template (#256) at
    the injection's exact parameters."""
    i = np.arange(16)
    lnmc = math.log(20.0) + i * math.log(2.0) / 15.0
    f0 = 0.014 + i * (0.002 / 15.0)
    LM, F0 = np.meshgrid(lnmc, f0, indexing="ij")
    mc = np.append(np.exp(LM.ravel()), TINY_INJECTION["mc"])
    f0v = np.append(F0.ravel(), TINY_INJECTION["f0"])
    n = mc.size
    p = TINY_INJECTION
    return Bank(mc=mc, eta=np.full(n, p["eta"]), f0=f0v,
                cos_theta=np.full(n, p["cos_theta"]), phi=np.full(n, p["phi"]),
                psi=np.full(n, p["psi"]), cos_iota=np.full(n, p["cos_iota"]))


def random_bank(n: int, cfg_id: int, mc_range=(10.0, 60.0), f0_range=(0.010, 0.040),
                eta: float | None = 0.25, stream: int = STREAM_BANK) -> Bank:
    """Mc log-uniform, f0 uniform, isotropic sky, uniform psi in [0, pi), cos iota uniform."""
    g = rng(cfg_id, stream)
    mc = np.exp(g.uniform(math.log(mc_range[0]), math.log(mc_range[1]), n))
    f0 = g.uniform(f0_range[0], f0_range[1], n)
    ct = g.uniform(-1.0, 1.0, n)
    ph = g.uniform(0.0, 2.0 * math.pi, n)
    psi = g.uniform(0.0, math.pi, n)
    ci = g.uniform(-1.0, 1.0, n)
    if eta is None:
        et = _q_to_eta(g.uniform(0.5, 1.0, n))
    else:
        et = np.full(n, eta)
    return Bank(mc=mc, eta=et, f0=f0, cos_theta=ct, phi=ph, psi=psi, cos_iota=ci)


def full_injections(n: int = 20, cfg_id: int = 2):
    """Injection parameters for the full-size workload and their target SNRs."""
    g = rng(cfg_id, STREAM_INJ)
    mc = np.exp(g.uniform(math.log(10.0), math.log(60.0), n))
    f0 = g.uniform(0.010, 0.040, n)
    eta = _q_to_eta(g.uniform(0.5, 1.0, n))
    snr = g.uniform(11.0, 20.0, n)
    ct = g.uniform(-1.0, 1.0, n)
    ph = g.uniform(0.0, 2.0 * math.pi, n)
    psi = g.uniform(0.0, math.pi, n)
    ci = g.uniform(-1.0, 1.0, n)
    phase = g.uniform(0.0, 2.0 * math.pi, n)
    return Bank(mc=mc, eta=eta, f0=f0, cos_theta=ct, phi=ph, psi=psi, cos_iota=ci, phase=phase), snr


def full_bank(n: int = 1_000_000, with_exact: bool = True) -> Bank:
    """Random bank of the full-size workload (+ the 20 exact-parameter templates)."""
    b = random_bank(n, FULL.cfg_id)
    if with_exact:
        inj, _ = full_injections()
        inj = inj.subset(np.arange(len(inj)))
        inj.phase = None
        b = Bank.concat(b, inj)
    return b


def batching_bank(n: int = 4_000_000) -> Bank:
    """Wide-range bank of the batching workload: Mc log-U[5, 100], f0 U[5, 50] mHz."""
    return random_bank(n, 4, mc_range=(5.0, 100.0), f0_range=(0.005, 0.050))


def subsample_indices(n_total: int, n_sub: int, must_include=(), cfg_id: int = 3) -> np.ndarray:
    """First n_sub indices of a seeded permutation, always including must_include."""
    g = rng(cfg_id, STREAM_BANK)
    perm = g.permutation(n_total)
    must = np.asarray(list(must_include), dtype=np.int64)
    rest = perm[~np.isin(perm, must)]
    return np.concatenate([must, rest[: max(0, n_sub - must.size)]])
