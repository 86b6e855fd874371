"""Exact reference quantities for tiny lattices, computed by brute-force enumeration.

Independent of the oracle: the couplings are turned into a dense symmetric
coupling matrix with numpy index arithmetic, and every one of the 2^n states is
scored with the quadratic form E = -1/2 s^T W s - h^T s (Eq. 1 / Eq. 8 of the
paper written as a matrix product).  Boltzmann weights follow Eq. (7).
"""
from __future__ import annotations

import numpy as np


def coupling_matrix(J, periodic):
    """Dense W[n, n] with W_ij = sum of couplings on bonds between i and j."""
    Lz, Ly, Lx, _ = J.shape
    n = Lx * Ly * Lz
    W = np.zeros((n, n), np.float64)
    z, y, x = np.meshgrid(np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    coords = [x, y, z]
    lens = [Lx, Ly, Lz]
    idx = (x + Lx * (y + Ly * z)).ravel()
    for a in range(3):
        L = lens[a]
        if L < 2:
            continue
        c2 = coords[a] + 1
        ok = c2 < L
        if (periodic >> a) & 1:
            ok = np.ones_like(ok)
            c2 = c2 % L
        nc = list(coords)
        nc[a] = c2
        nidx = (nc[0] + Lx * (nc[1] + Ly * nc[2])).ravel()
        Jv = J[..., a].ravel().astype(np.float64)
        m = ok.ravel()
        for i, j, v in zip(idx[m], nidx[m], Jv[m]):
            W[i, j] += v
            W[j, i] += v
    return W


def all_states(n):
    """All 2^n spin configurations as an int8 array [2^n, n] of +-1."""
    codes = np.arange(2 ** n, dtype=np.int64)
    bits = (codes[:, None] >> np.arange(n)) & 1
    return (2 * bits - 1).astype(np.int8)


def energies(W, h, states):
    s = states.astype(np.float64)
    E = -0.5 * np.einsum("si,ij,sj->s", s, W, s)
    if h is not None:
        E -= s @ h.astype(np.float64)
    return np.rint(E).astype(np.int64)


def boltzmann_energy_pmf(E_states, beta):
    """Exact P(E) under Eq. (7) at inverse temperature beta."""
    levels, inv = np.unique(E_states, return_inverse=True)
    w = np.exp(-beta * (E_states - E_states.min()))
    p = np.bincount(inv, weights=w)
    return levels, p / p.sum()


def chi2_pvalue(counts, probs, min_expected=5.0):
    """Pearson chi-square goodness of fit (sparse cells pooled)."""
    from scipy.stats import chi2

    counts = np.asarray(counts, np.float64)
    probs = np.asarray(probs, np.float64)
    N = counts.sum()
    exp = probs * N
    order = np.argsort(exp)
    c_acc = e_acc = 0.0
    obs, ex = [], []
    for i in order:
        c_acc += counts[i]
        e_acc += exp[i]
        if e_acc >= min_expected:
            obs.append(c_acc)
            ex.append(e_acc)
            c_acc = e_acc = 0.0
    if e_acc > 0 and ex:
        obs[-1] += c_acc
        ex[-1] += e_acc
    obs, ex = np.array(obs), np.array(ex)
    stat = ((obs - ex) ** 2 / ex).sum()
    dof = max(len(ex) - 1, 1)
    return float(chi2.sf(stat, dof)), float(stat), dof
