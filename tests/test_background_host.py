"""Host-side background fits (no GPU): tile assignment, the power-law tail and Gumbel maximum-likelihood
fits, and the false-alarm probabilities they give, checked against closed forms, scipy and samples drawn
from known distributions."""
import numpy as np
import pytest
from scipy import stats

from paper_2510_19047_amd import background as bg


def test_tile_ids_on_a_grid():
    mc_e = np.array([10.0, 20.0, 40.0])
    f0_e = np.array([0.01, 0.02, 0.03, 0.04])
    mc = np.array([10.0, 19.999, 20.0, 40.0, 9.99, 25.0, 25.0])
    f0 = np.array([0.01, 0.035, 0.02, 0.04, 0.02, 0.041, 0.0299])
    t = bg.tile_ids(mc, f0, mc_e, f0_e)
    assert t.dtype == np.int32
    # (0,0) (0,2) (1,1) (1,2: both upper edges closed) outside outside (1,2)
    assert t.tolist() == [0, 2, 4, 5, -1, -1, 4]


def test_power_law_fit_closed_form_and_recovery():
    # three tail samples at u, u e, u e^2: sum of logs 3, so delta = -1 - 3/3 = -2; q = 3/4
    u = 7.0
    fit = bg.fit_power_law([1.0, u, u * np.e, u * np.e ** 2], u)
    assert fit.delta == pytest.approx(-2.0, rel=1e-15)
    assert fit.q == 0.75 and fit.n_tail == 3
    # Pareto samples with density ~ x^-(a+1) above u: the MLE recovers delta = -(a+1)
    rng = np.random.default_rng(3)
    a = 3.5
    x = u * rng.uniform(size=20000) ** (-1.0 / a)
    fit = bg.fit_power_law(x, u)
    assert fit.delta == pytest.approx(-(a + 1.0), abs=5 * a / np.sqrt(x.size))
    # survival: q at the threshold, then (U/u)^(delta+1); capped at 1 below
    assert bg.fap_power_law(u, fit) == pytest.approx(fit.q)
    assert bg.fap_power_law(2 * u, fit) == pytest.approx(fit.q * 2.0 ** (fit.delta + 1.0))
    assert bg.fap_power_law(1e-3, fit) == 1.0
    with pytest.raises(ValueError):
        bg.fit_power_law([1.0, 2.0], 5.0)


def test_gumbel_fit_matches_scipy_and_recovers_parameters():
    rng = np.random.default_rng(4)
    mu, beta = 55.0, 3.2
    x = stats.gumbel_r.rvs(loc=mu, scale=beta, size=4000, random_state=rng)
    fit = bg.fit_gumbel(x)
    loc, scale = stats.gumbel_r.fit(x)
    assert fit.mu == pytest.approx(loc, rel=1e-6)
    assert fit.beta == pytest.approx(scale, rel=1e-5)
    assert abs(fit.mu - mu) < 5 * beta / np.sqrt(x.size) * 1.1
    assert abs(fit.beta - beta) < 5 * 0.78 * beta / np.sqrt(x.size)
    # the MLE equations hold at the fit
    z = (x - fit.mu) / fit.beta
    assert np.mean(np.exp(-z)) == pytest.approx(1.0, rel=1e-9)
    # survival function against scipy
    U = np.array([40.0, 55.0, 70.0, 120.0])
    np.testing.assert_allclose(bg.fap_gumbel(U, fit), stats.gumbel_r.sf(U, loc=fit.mu, scale=fit.beta),
                               rtol=1e-12)
    assert bg.fap_gumbel(fit.mu, fit) == pytest.approx(1.0 - np.exp(-1.0), rel=1e-15)


def test_background_fits_on_planted_maxima():
    """Maxima of many independent chi-square-like draws: the Gumbel fit is the optimistic (smaller) FAP and
    the power law the conservative one far in the tail."""
    rng = np.random.default_rng(5)
    B = bg.Background.__new__(bg.Background)
    B.n_tiles, B.rows, B.arg_rows = 4, [], []
    for _ in range(200):
        B.rows.append(rng.chisquare(64, size=(4, 500)).max(axis=1))
        B.arg_rows.append(np.zeros(4, np.int64))
    pl, gb = B.fits()
    assert pl.delta < -1.0 and gb.beta > 0.0
    hi = np.quantile(B.maxima, 0.999) * 1.5
    g, p = B.fap(hi)
    assert 0.0 <= g < p <= 1.0
    g1, p1 = B.fap(hi, tile=1)
    assert 0.0 <= g1 <= 1.0 and 0.0 <= p1 <= 1.0


def test_segment_ladder_rejects_bad_ladders():
    from paper_2510_19047_amd import search
    for bad in [(), (4, 2), (2, 4, 1), (8, 8, 1), (4, 0)]:
        with pytest.raises(ValueError):
            search.segment_ladder(None, None, None, ladder=bad)
