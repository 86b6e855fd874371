"""Colour maps (Methods, "Graph Coloring"): the library's DSATUR colouring and the checks on
given maps (host code, no GPU), and the oracle's sampler under colourings other than the
closed form."""
import numpy as np
import pytest

import oracle
from paper_2503_10302_amd import sg
from paper_2503_10302_amd.inputs import (diluted_couplings, ej_couplings, geometric_ladder,
                                         missing_spin_couplings)
from tests._exact import all_states, coupling_matrix, energies
from tests.test_oracle_sampling import boltzmann_energy_pmf, chi2_pvalue, _energy_hist

SEED = 0xC0105


def _edges(J, periodic):
    """Bonds with J != 0 as (j, nb) pairs, from the coupling array alone."""
    Lz, Ly, Lx = J.shape[:3]
    out = []
    for z in range(Lz):
        for y in range(Ly):
            for x in range(Lx):
                j = x + Lx * (y + Ly * z)
                for a, (L, c) in enumerate(((Lx, x), (Ly, y), (Lz, z))):
                    if L < 2 or J[z, y, x, a] == 0:
                        continue
                    if c == L - 1 and not (periodic >> a) & 1:
                        continue
                    xyz = [x, y, z]
                    xyz[a] = (xyz[a] + 1) % L
                    nb = xyz[0] + Lx * (xyz[1] + Ly * xyz[2])
                    if nb != j:
                        out.append((j, nb))
    return out


def _bipartite(n, edges):
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    side = [-1] * n
    for s in range(n):
        if side[s] >= 0:
            continue
        side[s] = 0
        stack = [s]
        while stack:
            v = stack.pop()
            for u in adj[v]:
                if side[u] < 0:
                    side[u] = 1 - side[v]
                    stack.append(u)
                elif side[u] == side[v]:
                    return False
    return True


CASES = [((8, 8, 8), 7, 0.0, 0), ((5, 5, 5), 7, 0.0, 0), ((15, 15, 12), 4, 0.0, 0),
         ((15, 15, 15), 7, 0.0, 0), ((7, 6, 5), 7, 0.55, 0), ((9, 9, 9), 7, 0.7, 0),
         ((6, 6, 6), 7, 0.3, 0), ((10, 10, 10), 3, 0.0, 1), ((3, 3, 3), 7, 0.0, 0),
         ((2, 2, 2), 7, 0.0, 0), ((1, 1, 6), 4, 0.0, 0), ((11, 4, 3), 5, 0.2, 3)]


def _case(shape, periodic, p_absent, missing, seed):
    if missing:
        return missing_spin_couplings(shape, periodic, seed, missing)
    if p_absent > 0:
        return diluted_couplings(shape, periodic, seed, p_absent)
    return ej_couplings(shape, periodic, seed)[0]


@pytest.mark.parametrize("shape,periodic,p_absent,missing", CASES)
def test_dsatur_colouring_is_proper_and_two_colours_on_bipartite_graphs(shape, periodic, p_absent,
                                                                         missing):
    """Every bond joins different colours (all bonds checked); DSATUR is exact on bipartite
    graphs (two colours, one for a graph without bonds) and needs three on the odd periodic
    cubes, which contain odd cycles."""
    J = _case(shape, periodic, p_absent, missing, 5)
    col, C = sg.dsatur((J, periodic, None))
    n = int(np.prod(shape))
    E = _edges(J, periodic)
    assert col.shape == (n,) and col.min() >= 0 and col.max() == C - 1 and C <= 4
    for a, b in E:
        assert col[a] != col[b], (a, b)
    if not E:
        assert C == 1
    elif _bipartite(n, E):
        assert C == 2
    else:
        assert C >= 3
    if shape == (15, 15, 15) or shape == (5, 5, 5):
        assert C in (3, 4)   # DSATUR is a heuristic off bipartite graphs (3 is optimal here)


def test_given_colour_maps_are_checked_before_device_work():
    J, _ = ej_couplings((4, 4, 4), 7, seed=1)
    beta = geometric_ladder(4)
    closed = (np.indices((4, 4, 4)).sum(axis=0) % 2).astype(np.int8).reshape(-1)   # (x+y+z) mod 2
    bad = closed.copy()
    bad[1] = bad[0]                                    # sites 0 and 1 are bonded along x
    for m in (bad, np.full(64, 4, np.int8), np.full(64, -1, np.int8)):
        with pytest.raises(sg.SGError) as e:
            sg.apt([(J, 7, None)], beta, 1, 2, colours=[m])
        assert e.value.code == sg.SG_EINVAL
    J0 = J.copy()                                      # site 0 without any bond: any colour will do
    J0[0, 0, 0, :] = 0
    J0[0, 0, 3, 0] = J0[0, 3, 0, 1] = J0[3, 0, 0, 2] = 0
    lone = closed.copy()
    lone[0] = 1 - lone[0]
    try:
        sg.apt([(J0, 7, None)], beta, 1, 2, colours=[lone])
    except sg.SGError as e:
        assert e.code == sg.SG_EHIP                    # accepted; fails later only for want of a GPU


def _four_colouring(shape):
    """A proper four-colouring of an even periodic box: the checkerboard with each class split
    at random in two."""
    base = (np.indices(shape[::-1]).sum(axis=0) % 2).reshape(-1)
    rng = np.random.default_rng(3)
    return (base + 2 * (rng.random(base.size) < 0.5)).astype(np.int8)


@pytest.mark.parametrize("colouring", ["dsatur", "four"])
def test_oracle_samples_boltzmann_under_other_colourings(colouring):
    """The coloured Gibbs sweep samples Eq. (7) under any proper colouring, not only the closed
    form: chi-square of sampled energies against exact enumeration (18 spins), failing against
    a perturbed beta."""
    shape = (2, 3, 3) if colouring == "dsatur" else (2, 2, 4)
    per = 0 if colouring == "dsatur" else 7
    J = _case(shape, per, 0.2 if colouring == "dsatur" else 0.0, 0, 8)
    if colouring == "dsatur":
        col, _ = sg.dsatur((J, per, None))
    else:
        col = _four_colouring(shape)
        for a, b in _edges(J, per):
            assert col[a] != col[b]
    lat = oracle.Lattice(J, per, None, col)
    assert oracle.n_colours(lat) == int(col.max()) + 1
    Es = energies(coupling_matrix(J, per), None, all_states(lat.n))
    spins = oracle.apt_init(lat, 0, 4, SEED)
    beta = np.full(4, 0.6)
    samples = []
    for t in range(6000):
        oracle.apt_sweep(lat, 0, beta, SEED, t, spins)
        if t >= 50:
            samples += [oracle.energy(lat, s) for s in spins]
    levels, p = boltzmann_energy_pmf(Es, 0.6)
    cnt = _energy_hist(levels, np.array(samples))
    assert chi2_pvalue(cnt, p)[0] > 1e-4
    _, pw = boltzmann_energy_pmf(Es, 0.8)
    assert chi2_pvalue(cnt, pw)[0] < 1e-6


@pytest.mark.parametrize("M", [4, 6, 5])
def test_oracle_trotter_colouring_with_a_map_is_proper(M):
    J = diluted_couplings((5, 5, 4), 7, seed=9, p_absent=0.6)
    col, C = sg.dsatur((J, 7, None))
    lat = oracle.Lattice(J, 7, None, col)
    E = _edges(J, 7)
    for k in range(M):
        for a, b in E:
            assert oracle.colour(lat, a, M, k) != oracle.colour(lat, b, M, k)
        for j in range(lat.n):
            for kk in ((k + 1) % M, (k - 1) % M):
                assert oracle.colour(lat, j, M, kk) != oracle.colour(lat, j, M, k)
