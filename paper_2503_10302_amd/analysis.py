"""Analysis of Monte Carlo results returned by the library (host code, no Monte Carlo
arithmetic): residual energy per spin (Eq. 2), the power-law slope kappa_f (Eq. 3) with a
confidence interval, bootstrap confidence intervals of means across instances, the extreme-value
statistics of the Supplementary EVT section (median and mean of the minimum of P Gaussian
energies, the residual-energy prediction and the self-consistent block size of the modified
EVT), the correlation along the Trotter direction, and a finite-size-scaling collapse measure.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special, stats


def residual(E, E0, n):
    """Eq. (2) before averaging: (E - E0) / n per run."""
    return (np.asarray(E, np.float64) - np.asarray(E0, np.float64)) / n


def bootstrap_ci(x, n_boot=2000, level=0.95, seed=0):
    """Percentile bootstrap confidence interval of the mean of x (resampling with replacement
    across instances, as the paper's error bars)."""
    x = np.asarray(x, np.float64)
    rng = np.random.default_rng(seed)
    means = x[rng.integers(0, x.size, size=(n_boot, x.size))].mean(axis=1)
    lo, hi = np.quantile(means, [(1 - level) / 2, (1 + level) / 2])
    return float(lo), float(hi)


def power_law_fit(t, rho, level=0.95):
    """Eq. (3): rho = A t^(-kappa), least squares in log-log.  Returns kappa, A and the
    confidence interval of kappa from the slope's standard error (Student t)."""
    lt, lr = np.log(np.asarray(t, np.float64)), np.log(np.asarray(rho, np.float64))
    n = lt.size
    X = np.stack([np.ones(n), lt], axis=1)
    coef, res, _, _ = np.linalg.lstsq(X, lr, rcond=None)
    kappa, A = -coef[1], math.exp(coef[0])
    if n > 2:
        resid = lr - X @ coef
        s2 = float(resid @ resid) / (n - 2)
        se = math.sqrt(s2 / float(((lt - lt.mean()) ** 2).sum()))
        h = stats.t.ppf((1 + level) / 2, n - 2) * se
    else:
        h = float("nan")
    return {"kappa": float(kappa), "A": A, "ci": (float(kappa - h), float(kappa + h))}


# ---- extreme-value statistics (Supplementary EVT section) -------------------------------
def evt_median_min(mu, sigma, P):
    """Median of the minimum of P i.i.d. Gaussians N(mu, sigma): F_P(x) = 1 - (1 - F(x))^P = 1/2
    gives x_p = mu + sqrt(2) sigma erfc^-1(2^((P - 1) / P))."""
    return mu + math.sqrt(2.0) * sigma * special.erfcinv(2.0 ** ((P - 1.0) / P))


def evt_median_asymptotic(mu, sigma, P):
    """Large-P expansion of x_p: mu - sigma sqrt(c + ln2/P + 2 lnP - ln(c + ln2/P + 2 lnP)),
    c = ln(2 / (pi (ln 4)^2))."""
    c = math.log(2.0 / (math.pi * math.log(4.0) ** 2))
    u = c + math.log(2.0) / P + 2.0 * math.log(P)
    return mu - sigma * math.sqrt(u - math.log(u))


def evt_median_textbook(mu, sigma, P):
    """The leading term: x_p ~ mu - sigma sqrt(2 ln P)."""
    return mu - sigma * math.sqrt(2.0 * math.log(P))


def evt_mean_min(mu, sigma, P):
    """Expected minimum of P i.i.d. Gaussians: the integral of x dF_P(x), F_P = 1 - (1-F)^P,
    evaluated numerically in the standardised variable."""
    def integrand(z):
        return z * P * stats.norm.pdf(z) * stats.norm.sf(z) ** (P - 1)
    val, _ = integrate.quad(integrand, -np.inf, np.inf, limit=200)
    return mu + sigma * val


def evt_rho(a, b, P):
    """Residual energy predicted for the best of P independent runs whose residual energies
    have mean a and standard deviation b: a + sqrt(2) b erfc^-1(2^((P - 1) / P))."""
    return a + math.sqrt(2.0) * b * special.erfcinv(2.0 ** ((P - 1.0) / P))


def block_minima(E, B):
    """Minimum over consecutive blocks of B slices along the last axis (length divisible by B)."""
    E = np.asarray(E)
    M = E.shape[-1]
    if M % B:
        raise ValueError("block size must divide the number of slices")
    return E.reshape(E.shape[:-1] + (M // B, B)).min(axis=-1)


def evt_prediction(best, E0, n, P):
    """Conventional EVT for one annealing time: best[i][r] = lowest energy of independent run r of
    instance i.  Per instance the mean and standard deviation of the runs' residual energies; a,
    b = their averages over instances; returns (predicted rho for the best of P runs, measured rho
    = mean over instances of the mean over disjoint groups of P runs of the group's best)."""
    res = residual(best, np.asarray(E0)[:, None], n)
    a = float(res.mean(axis=1).mean())
    b = float(res.std(axis=1, ddof=1).mean())
    R = res.shape[1] // P * P
    meas = float(res[:, :R].reshape(res.shape[0], -1, P).min(axis=2).mean())
    return evt_rho(a, b, P), meas, a, b


def block_size_fit(slice_E, E0, n, sizes=None, tol=0.01):
    """Modified EVT (self-consistent block size): slice_E[i][r][k] final energies of slice k of
    independent replica r of instance i (M slices on a Trotter ring).  For each candidate block
    size B < M the minima of blocks of B consecutive slices give, per instance, the mean and
    standard deviation of their residual energies; with a, b their averages and P = M / B blocks,
    evt_rho(a, b, P) predicts the residual energy of the best slice, compared with the measured
    one (mean over instances and replicas).  Blocks smaller than the correlation length treat
    correlated slices as independent and predict too low a residual; the block size is the
    smallest B whose prediction comes within a relative `tol` of the measurement (B = M would
    reproduce it trivially and is not a candidate).  Returns the table, that B, and the B whose
    prediction is closest."""
    slice_E = np.asarray(slice_E)
    M = slice_E.shape[-1]
    sizes = [B for B in (sizes or range(1, M)) if M % B == 0 and B < M]
    meas = float(residual(slice_E.min(axis=-1), np.asarray(E0)[:, None], n).mean())
    table = {}
    for B in sizes:
        bm = residual(block_minima(slice_E, B), np.asarray(E0)[:, None, None], n)
        flat = bm.reshape(bm.shape[0], -1)
        a = float(flat.mean(axis=1).mean())
        b = float(flat.std(axis=1, ddof=1).mean()) if flat.shape[1] > 1 else 0.0
        table[B] = {"P": M // B, "a": a, "b": b, "predicted": evt_rho(a, b, M // B)}
    reach = [B for B in sizes if table[B]["predicted"] >= meas - tol * abs(meas)]
    closest = min(table, key=lambda B: abs(table[B]["predicted"] - meas))
    return {"measured": meas, "block_size": reach[0] if reach else sizes[-1], "closest": closest,
            "table": table}


def trotter_correlation(agree, n):
    """C_k = (1/n) sum_i s_{i,0} s_{i,k} from agreement counts [..., M], averaged over the
    leading axes (instances, replicas)."""
    a = np.asarray(agree, np.float64)
    C = (2.0 * a - n) / n
    return C.reshape(-1, a.shape[-1]).mean(axis=0)


def collapse_spread(curves, mu, b):
    """Finite-size-scaling collapse (Supplementary FSS figures): for curves {L: (t, rho)} the
    rescaled points (t L^-mu, rho L^b) of every size are interpolated in log-log onto a common
    range of the rescaled time; returns the mean over that range of the standard deviation of
    log(rho L^b) across sizes (small when the curves collapse)."""
    xs, ys = [], []
    for L, (t, rho) in curves.items():
        t, rho = np.asarray(t, np.float64), np.asarray(rho, np.float64)
        ok = rho > 0
        xs.append(np.log(t[ok] * float(L) ** -mu))
        ys.append(np.log(rho[ok] * float(L) ** b))
    lo = max(x.min() for x in xs)
    hi = min(x.max() for x in xs)
    if not hi > lo:
        return float("inf")
    grid = np.linspace(lo, hi, 25)
    vals = np.stack([np.interp(grid, x, y) for x, y in zip(xs, ys)])
    return float(vals.std(axis=0).mean())
