"""Data transform: tranche-wise windowed DFT and whitening.

Paper passages followed: each tranche is Tukey-windowed (shape 0.1) and
Fourier transformed once (Sec. "Implementation details"); the PSD may differ
from tranche to tranche (locally stationary noise, Sec. "Search extension to
data with gaps"); tranches that overlap a gap are left out of Eq. (inner-tf).

Readings fixed here:
* Tranche m holds samples mM .. mM + M - 1; its DFT uses the local time
  origin: X_mk = sum_j w_j x_{mM+j} exp(-2 pi i j k / M), k = 0..M/2.
* The Tukey window is scipy's symmetric one (M points, shape alpha);
  alpha = 0 is the rectangular window.
* Pixels are whitened to unit variance for stationary noise of one-sided PSD
  S_m(f) = mu_m S0(f):  D_mk = X_mk sqrt(2 dt / (M W2 S_m(f_k))), W2 = mean(w^2).
  Excluded tranches are zero.  The companion per-bin and per-tranche
  template weights are u_k = 1/sqrt(S0(f_k)) and w_m = 1/sqrt(mu_m) (0 when
  excluded).  DC and Nyquist are never used by the statistic.
* Layout of the pixel store: [C][K][Nt] complex, K = M/2 + 1 (tranches
  contiguous within a frequency layer).
* A PSD that varies between tranches in a general way (not mu_m S0(f)) is
  given as S[K, Nt] = S_m(f_k); the pixels are whitened by it pixel by pixel,
  D_mk = X_mk sqrt(2 dt / (M W2 S_m(f_k))), and the template weight of pixel
  (m, k) is keep_m / sqrt(S_m(f_k)) (``transform_tf``).
"""
from __future__ import annotations

import numpy as np


def tukey(M: int, alpha: float) -> np.ndarray:
    if alpha <= 0.0:
        return np.ones(M)
    from scipy.signal.windows import tukey as _tk
    return _tk(M, alpha)


def dft_matrix(M: int) -> np.ndarray:
    """E[k, j] = exp(-2 pi i (j k mod M) / M) for k = 0..M/2, exact integer phase index."""
    k = np.arange(M // 2 + 1, dtype=np.int64)[:, None]
    j = np.arange(M, dtype=np.int64)[None, :]
    idx = (j * k) % M
    return np.exp(-2j * np.pi * idx / M)


def tranche_dft(x: np.ndarray, M: int, alpha: float, method: str = "direct") -> np.ndarray:
    """Windowed DFT of every tranche of one channel: returns X[K, Nt] (complex128).

    method 'direct' is the exact-index naive DFT; 'rfft' uses numpy.fft.rfft.
    """
    x = np.asarray(x, dtype=np.float64 if not np.iscomplexobj(x) else np.complex128)
    Nt = x.size // M
    w = tukey(M, alpha)
    seg = x[: Nt * M].reshape(Nt, M) * w[None, :]
    if method == "direct":
        E = dft_matrix(M)
        return E @ seg.T
    if np.iscomplexobj(seg):
        full = np.fft.fft(seg, axis=1)
        return full[:, : M // 2 + 1].T
    return np.fft.rfft(seg, axis=1).T


def whitening(M: int, dt: float, alpha: float, psd0: np.ndarray, mu: np.ndarray, keep: np.ndarray):
    """(scale[K, Nt], u[K], w[Nt]) for the whitening described above."""
    w = tukey(M, alpha)
    W2 = float(np.mean(w * w))
    keep = np.asarray(keep, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    scale = np.sqrt(2.0 * dt / (M * W2 * psd0[:, None] * mu[None, :])) * keep[None, :]
    u = 1.0 / np.sqrt(psd0)
    wm = np.where(keep > 0, 1.0 / np.sqrt(mu), 0.0)
    return scale, u, wm


def transform(x: np.ndarray, grid, psd0: np.ndarray, mu: np.ndarray, keep: np.ndarray,
              alpha: float = 0.1, method: str = "direct"):
    """Pixels [C][K][Nt] complex128 plus (u[K], w[Nt]) from time-domain data [C][N]."""
    M = grid.tranche_len
    x = np.atleast_2d(x)
    scale, u, wm = whitening(M, grid.dt, alpha, psd0, mu, keep)
    pix = np.empty((x.shape[0], M // 2 + 1, grid.n_tranches), dtype=np.complex128)
    for c in range(x.shape[0]):
        pix[c] = tranche_dft(x[c], M, alpha, method) * scale
    return pix, u, wm


def whitening_tf(M: int, dt: float, alpha: float, psd_tf: np.ndarray, keep: np.ndarray):
    """(scale[K, Nt], weight[K, Nt]) for a PSD S_m(f_k) given pixel by pixel (psd_tf[K, Nt])."""
    w = tukey(M, alpha)
    W2 = float(np.mean(w * w))
    keep = np.asarray(keep, dtype=np.float64)
    S = np.asarray(psd_tf, dtype=np.float64)
    if S.shape != (M // 2 + 1, keep.shape[0]):
        raise ValueError("psd_tf must be [M/2 + 1, Nt]")
    scale = np.sqrt(2.0 * dt / (M * W2 * S)) * keep[None, :]
    weight = np.where(keep[None, :] > 0, 1.0 / np.sqrt(S), 0.0)
    return scale, weight


def transform_tf(x: np.ndarray, grid, psd_tf: np.ndarray, keep: np.ndarray, alpha: float = 0.1,
                 method: str = "direct"):
    """Pixels [C][K][Nt] complex128 plus the per-pixel template weights [K][Nt] for a PSD that differs
    from tranche to tranche in a general way (psd_tf[K, Nt] = S_m(f_k))."""
    M = grid.tranche_len
    x = np.atleast_2d(x)
    scale, weight = whitening_tf(M, grid.dt, alpha, psd_tf, keep)
    pix = np.empty((x.shape[0], M // 2 + 1, grid.n_tranches), dtype=np.complex128)
    for c in range(x.shape[0]):
        pix[c] = tranche_dft(x[c], M, alpha, method) * scale
    return pix, weight
