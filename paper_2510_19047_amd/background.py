"""Background distribution of the statistic and false-alarm probabilities of candidates.

Paper Sec. "Results" (false-alarm probabilities): the background is built empirically from noise-only
realisations, one search per realisation, keeping the largest statistic per parameter tile; its tail is
extrapolated with a power law p0(U) ~ U^delta (conservative, the upper FAP bound) and with a Gumbel
distribution of location mu and scale beta (optimistic, the lower bound).  The FAP of a candidate with
statistic U is the probability that the search of a noise-only data set returns a value >= U in the tile.

Here a realisation's "search" is the bank evaluation (``bank_statistic`` or a ``RealisationGraph``
replay), the per-tile maxima come from ``tile_max`` on the device, and the fits are host-side maximum
likelihood on the few hundred maxima that result.  Nothing here computes any part of the statistic.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import tile_max


def tile_ids(mc: np.ndarray, f0: np.ndarray, mc_edges: np.ndarray, f0_edges: np.ndarray) -> np.ndarray:
    """Tile index i_mc * (len(f0_edges) - 1) + i_f0 of each template on a (Mc, f0) grid of bin edges;
    -1 outside the grid.  Intervals are closed on the left, open on the right (the last one closed)."""
    mc_edges, f0_edges = np.asarray(mc_edges, np.float64), np.asarray(f0_edges, np.float64)
    nm, nf = len(mc_edges) - 1, len(f0_edges) - 1
    im = np.searchsorted(mc_edges, mc, side="right") - 1
    jf = np.searchsorted(f0_edges, f0, side="right") - 1
    im = np.where(mc == mc_edges[-1], nm - 1, im)
    jf = np.where(f0 == f0_edges[-1], nf - 1, jf)
    ok = (im >= 0) & (im < nm) & (jf >= 0) & (jf < nf)
    return np.where(ok, im * nf + jf, -1).astype(np.int32)


@dataclass
class PowerLawTail:
    """p0(U) proportional to U^delta for U >= u; q = fraction of the samples at or above u."""
    u: float
    delta: float
    q: float
    n_tail: int


@dataclass
class GumbelFit:
    """p0(U) = exp(-(z + exp(-z))) / beta with z = (U - mu) / beta."""
    mu: float
    beta: float


def fit_power_law(x, u: float) -> PowerLawTail:
    """Maximum-likelihood exponent of a power-law tail above u (the Hill estimator):
    delta = -1 - k / sum(ln(x_i / u)) over the k samples x_i >= u."""
    x = np.asarray(x, np.float64)
    if not u > 0.0:
        raise ValueError("the tail threshold must be positive")
    tail = x[x >= u]
    s = float(np.sum(np.log(tail / u)))
    if tail.size < 2 or not s > 0.0:
        raise ValueError("need at least two tail samples above the threshold")
    return PowerLawTail(float(u), -1.0 - tail.size / s, tail.size / x.size, int(tail.size))


def fit_gumbel(x) -> GumbelFit:
    """Maximum-likelihood Gumbel (maximum) location and scale.  beta solves
    beta = mean(x) - sum(x_i w_i) / sum(w_i), w_i = exp(-x_i / beta); mu = -beta ln(mean(exp(-x_i / beta)))."""
    from scipy.optimize import brentq
    x = np.asarray(x, np.float64)
    if x.size < 2 or not np.ptp(x) > 0.0:
        raise ValueError("need at least two distinct samples")
    x0 = x.min()
    y = x - x0  # shift for the exponentials; the scale equation is shift-invariant

    def g(beta):
        w = np.exp(-(y - y.min()) / beta)
        return y.mean() - np.sum(y * w) / np.sum(w) - beta

    sd = float(np.std(y))
    lo, hi = 1e-6 * sd, 10.0 * sd
    beta = brentq(g, lo, hi, xtol=1e-14 * sd, rtol=1e-14, maxiter=400)
    mu = x0 - beta * (np.log(np.mean(np.exp(-(y - y.min()) / beta))) - y.min() / beta)
    return GumbelFit(float(mu), float(beta))


def fap_power_law(U, fit: PowerLawTail):
    """P(max >= U) from the power-law tail: q (U / u)^(delta + 1), capped at 1."""
    U = np.asarray(U, np.float64)
    return np.minimum(1.0, fit.q * np.power(np.maximum(U, 1e-300) / fit.u, fit.delta + 1.0))


def fap_gumbel(U, fit: GumbelFit):
    """P(max >= U) = 1 - exp(-exp(-(U - mu) / beta))."""
    z = (np.asarray(U, np.float64) - fit.mu) / fit.beta
    return -np.expm1(-np.exp(-z))


class Background:
    """Per-tile maxima of the statistic over noise-only realisations.

    ``add(stat)`` takes one realisation's bank statistic (device, float64) and records its per-tile
    maxima (``tile_max`` on the device).  ``maxima`` is [R][n_tiles] (``argmax`` the template index,
    -1 for a tile without templates); ``fits`` gives the power-law and Gumbel tails of one tile's
    maxima, or of all non-empty tiles pooled.
    """

    def __init__(self, tile: np.ndarray, n_tiles: int, device="cuda"):
        self.n_tiles = int(n_tiles)
        self.tile = torch.from_numpy(np.ascontiguousarray(tile, dtype=np.int32)).to(device)
        self._out = None
        self.rows: list[np.ndarray] = []
        self.arg_rows: list[np.ndarray] = []

    def add(self, stat: torch.Tensor) -> np.ndarray:
        self._out = tile_max(stat, self.tile, self.n_tiles, out=self._out)
        row = self._out[0].cpu().numpy().copy()
        self.rows.append(row)
        self.arg_rows.append(self._out[1].cpu().numpy().copy())
        return row

    @property
    def maxima(self) -> np.ndarray:
        return np.stack(self.rows) if self.rows else np.zeros((0, self.n_tiles))

    @property
    def argmax(self) -> np.ndarray:
        return np.stack(self.arg_rows) if self.arg_rows else np.zeros((0, self.n_tiles), np.int64)

    def fits(self, tile: int | None = None, tail_fraction: float = 0.5):
        """(PowerLawTail, GumbelFit) of one tile's maxima over the realisations, or of every non-empty
        tile's maxima pooled (tile=None).  The power law is fitted above the (1 - tail_fraction) quantile."""
        mx, arg = self.maxima, self.argmax
        if tile is not None:
            mx, arg = mx[:, tile], arg[:, tile]
        x = np.asarray(mx, np.float64)[np.asarray(arg) >= 0]
        u = float(np.quantile(x, 1.0 - tail_fraction))
        return fit_power_law(x, u), fit_gumbel(x)

    def fap(self, U, tile: int | None = None, tail_fraction: float = 0.5):
        """(optimistic, conservative) false-alarm probabilities of a statistic value U: the Gumbel and
        the power-law extrapolations of the background."""
        pl, gb = self.fits(tile, tail_fraction)
        return fap_gumbel(U, gb), fap_power_law(U, pl)
