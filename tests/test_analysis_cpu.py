"""Pins for the analysis formulas (Supplementary EVT section; Eqs. 2-3): each is checked against
something other than itself -- exact order statistics of the normal law, the known means of the
minimum of two and three standard normals, Monte Carlo, exact power laws."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2503_10302_amd import analysis as A


@pytest.mark.parametrize("P", [1, 2, 3, 10, 50, 1000])
def test_evt_median_equals_order_statistic(P):
    """x_p = mu + sqrt(2) sigma erfc^-1(2^((P-1)/P)) is the median of the minimum of P normals:
    Phi^-1(1 - 2^(-1/P)) from the order-statistics CDF, and a Monte Carlo median."""
    mu, sigma = -1.7, 0.3
    exact = mu + sigma * stats.norm.ppf(1.0 - 2.0 ** (-1.0 / P))
    assert abs(A.evt_median_min(mu, sigma, P) - exact) < 1e-12
    rng = np.random.default_rng(P)
    mins = (mu + sigma * rng.standard_normal((20000, P))).min(axis=1)
    se = 1.253 * mins.std() / math.sqrt(mins.size)      # standard error of a sample median
    assert abs(np.median(mins) - A.evt_median_min(mu, sigma, P)) < 5 * se


def test_evt_mean_known_values():
    """E[min of 2 standard normals] = -1/sqrt(pi), of 3 = -3/(2 sqrt(pi)); P = 1 gives mu."""
    assert abs(A.evt_mean_min(0.0, 1.0, 2) + 1.0 / math.sqrt(math.pi)) < 1e-9
    assert abs(A.evt_mean_min(0.0, 1.0, 3) + 1.5 / math.sqrt(math.pi)) < 1e-9
    assert abs(A.evt_mean_min(2.0, 3.0, 1) - 2.0) < 1e-9
    rng = np.random.default_rng(4)
    mins = rng.standard_normal((200000, 50)).min(axis=1)
    assert abs(mins.mean() - A.evt_mean_min(0.0, 1.0, 50)) < 5 * mins.std() / math.sqrt(mins.size)


def test_evt_asymptotics():
    """The expansion approaches the exact median as P grows and beats the textbook term; the
    textbook term's relative error falls towards zero only slowly."""
    errs = []
    for P in (10, 100, 10 ** 4, 10 ** 6):
        ex = A.evt_median_min(0.0, 1.0, P)
        errs.append(abs(A.evt_median_asymptotic(0.0, 1.0, P) - ex) / abs(ex))
        assert abs(A.evt_median_asymptotic(0.0, 1.0, P) - ex) < abs(A.evt_median_textbook(0.0, 1.0, P) - ex)
    assert errs[-1] < 2e-3 and errs == sorted(errs, reverse=True)
    assert abs(A.evt_median_textbook(0.0, 1.0, 10 ** 12) / A.evt_median_min(0.0, 1.0, 10 ** 12) - 1) < 0.05


def test_evt_prediction_on_gaussian_runs():
    """Runs whose energies are Gaussian: the predicted residual of the best of P runs matches the
    measured one (disjoint groups)."""
    rng = np.random.default_rng(5)
    n, E0 = 1000, np.full(40, -1700.0)
    best = -1690.0 + 4.0 * rng.standard_normal((40, 4096))
    for P in (1, 4, 16, 64):
        pred, meas, a, b = A.evt_prediction(best, E0, n, P)
        assert abs(a - 0.01) < 1e-3 and abs(b - 0.004) < 2e-4
        assert abs(pred - meas) < 3e-4, (P, pred, meas)


def test_block_size_fit_recovers_independent_blocks():
    """Slices that are copies within blocks of 4 and independent Gaussians across blocks: blocks
    of 1 and 2 slices treat copies as independent and predict too low a residual energy; the
    self-consistent block size is 4."""
    rng = np.random.default_rng(6)
    ind = -995.0 + 5.0 * rng.standard_normal((24, 200, 8))
    slice_E = np.repeat(ind, 4, axis=2)           # M = 32, blocks of 4 identical slices
    fit = A.block_size_fit(slice_E, np.full(24, -1010.0), 1000)
    assert fit["block_size"] == 4
    assert fit["table"][4]["P"] == 8 and 32 not in fit["table"]
    assert fit["table"][1]["predicted"] < fit["table"][2]["predicted"] < fit["measured"]


def test_power_law_fit_and_bootstrap():
    t = np.array([50, 100, 200, 500, 1000, 3000.0])
    rho = 0.3 * t ** -0.647
    f = A.power_law_fit(t, rho)
    assert abs(f["kappa"] - 0.647) < 1e-12 and abs(f["A"] - 0.3) < 1e-12
    rng = np.random.default_rng(7)
    hits = 0
    for k in range(200):
        noisy = rho * np.exp(0.05 * rng.standard_normal(t.size))
        lo, hi = A.power_law_fit(t, noisy)["ci"]
        hits += lo <= 0.647 <= hi
    assert 180 <= hits <= 200                     # about 95 % coverage
    x = rng.normal(2.0, 1.0, 300)
    lo, hi = A.bootstrap_ci(x)
    assert lo < x.mean() < hi and abs((hi - lo) - 2 * 1.96 / math.sqrt(300)) < 0.05
    assert A.bootstrap_ci(np.full(10, 3.0)) == (3.0, 3.0)


def test_trotter_correlation_and_collapse():
    n = 100
    agree = np.array([[[100, 75, 50, 25]]])
    assert np.allclose(A.trotter_correlation(agree, n), [1.0, 0.5, 0.0, -0.5])
    t = np.logspace(1, 4, 12)
    mu, b = 2.0, 3.0
    curves = {L: (t * L ** mu, 0.2 * (t ** -0.6) * L ** -b) for L in (6, 8, 10, 12)}
    assert A.collapse_spread(curves, mu, b) < 1e-9
    assert A.collapse_spread(curves, mu + 1.0, b) > 0.1
