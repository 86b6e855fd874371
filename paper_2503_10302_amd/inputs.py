"""Seeded synthetic inputs: +-J Edwards-Anderson instances, beta ladders, Gamma ramps.

This module holds no arithmetic of the Monte Carlo method itself.  It only draws
problem inputs with the structure of the paper's workloads (Eq. 1: nearest-
neighbour couplings on a cubic lattice, each +1 or -1 with equal probability;
Methods, "Annealing Schedule of DT-SQA": a linear transverse-field ramp).  The
paper's own instances are not available, so these stand in for them.  Both the
product library's callers and the test oracle take their inputs from here.
"""
from __future__ import annotations

import numpy as np


def ej_couplings(shape, periodic=7, seed=0, h_max=0):
    """+-1 couplings J[Lz, Ly, Lx, 3] (bond to +x, +y, +z) and fields h[n].

    Bonds that would cross an open boundary are set to 0 (absent).  With
    ``h_max > 0`` the fields are uniform integers in [-h_max, h_max];
    otherwise h is None (all zero).
    """
    if np.isscalar(shape):
        shape = (int(shape),) * 3
    Lx, Ly, Lz = (int(v) for v in shape)
    rng = np.random.default_rng(np.random.SeedSequence([0x5EED, int(seed)]))
    J = np.where(rng.random((Lz, Ly, Lx, 3)) < 0.5, 1, -1).astype(np.int8)
    for axis, L in enumerate((Lx, Ly, Lz)):
        if not (periodic >> axis) & 1 or L < 2:
            idx = [slice(None)] * 3
            idx[2 - axis] = L - 1  # array axes are (z, y, x)
            J[tuple(idx) + (axis,)] = 0
    h = None
    if h_max > 0:
        h = rng.integers(-h_max, h_max + 1, size=Lx * Ly * Lz).astype(np.int8)
    return J, h


def diluted_couplings(shape, periodic=7, seed=0, p_absent=0.1):
    """+-1 couplings with a random fraction of bonds removed (J = 0)."""
    J, _ = ej_couplings(shape, periodic, seed)
    rng = np.random.default_rng(np.random.SeedSequence([0xD11, int(seed)]))
    J[rng.random(J.shape) < p_absent] = 0
    return J


def geometric_ladder(n=32, lo=0.2, hi=3.0):
    """n inverse temperatures geometric in [lo, hi] (ascending)."""
    k = np.arange(n, dtype=np.float64)
    return lo * (hi / lo) ** (k / (n - 1))


def linear_gamma(n_steps, start=3.0, end=0.01):
    """Transverse field ramped linearly from start to end, both included."""
    if n_steps == 1:
        return np.array([start], np.float64)
    t = np.arange(n_steps, dtype=np.float64)
    return start + (end - start) * t / (n_steps - 1)


def mixed_sizes(n_inst, sizes=(6, 8, 10, 12, 15)):
    """Round-robin lattice sizes for a batch of instances."""
    return [sizes[i % len(sizes)] for i in range(n_inst)]


def missing_spin_couplings(shape, periodic=7, seed=0, n_missing=1):
    """+-1 couplings with `n_missing` randomly chosen sites removed: every bond of a missing
    site is 0, so it is isolated (the paper's L = 10 instances have 999 of 1000 spins)."""
    J, _ = ej_couplings(shape, periodic, seed)
    if np.isscalar(shape):
        shape = (int(shape),) * 3
    Lx, Ly, Lz = (int(v) for v in shape)
    rng = np.random.default_rng(np.random.SeedSequence([0x5717, int(seed)]))
    for j in rng.choice(Lx * Ly * Lz, size=n_missing, replace=False):
        x, y, z = j % Lx, (j // Lx) % Ly, j // (Lx * Ly)
        J[z, y, x, :] = 0
        J[z, y, (x - 1) % Lx, 0] = 0
        J[z, (y - 1) % Ly, x, 1] = 0
        J[(z - 1) % Lz, y, x, 2] = 0
    return J
