"""Distributional pins: the oracle's Markov chains sample the laws the paper states.

 * Gibbs sweeps (Eqs. 5-6) leave the Boltzmann law (Eq. 7) invariant: chi-square of
   sampled energies and states against brute-force enumeration of every state.
 * Replica exchange (Eq. 4) keeps each temperature's marginal Boltzmann and its
   acceptance frequency is min(1, exp(dbeta dE)).
 * ICM (Algorithm S2, ICMop) keeps E1 + E2, flips exactly the overlap cluster of
   the chosen seed, and keeps the product law of two equal-temperature replicas.
 * DT-SQA sweeps (Supplementary Eqs. S.1-S.3) sample exp(-beta H_C) of the
   replicated lattice; large Gamma decouples slices into heat baths at beta/M.
 * The adaptive ladder follows beta_{t+1} = beta_t + alpha / sigma_E with the
   closed-form sigma_E of independent spins, and its swap acceptance is close to
   erfc(alpha / 2) for near-Gaussian energies.
Each test also checks its own power: the same samples must fail against a law
with a perturbed inverse temperature.
"""
import math

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components
from scipy.special import erfc

import oracle
from paper_2503_10302_amd.inputs import ej_couplings
from tests._exact import all_states, boltzmann_energy_pmf, chi2_pvalue, coupling_matrix, energies

SEED = 0xC0FFEE


def _energy_hist(levels, samples):
    pos = np.searchsorted(levels, samples)
    assert np.all(levels[pos] == samples)
    return np.bincount(pos, minlength=levels.size)


@pytest.mark.parametrize("shape,periodic,hmax", [((2, 2, 3), 4, 0), ((4, 4, 1), 3, 0), ((2, 3, 3), 0, 1)])
def test_gibbs_sweeps_sample_boltzmann(shape, periodic, hmax):
    J, h = ej_couplings(shape, periodic, seed=11, h_max=hmax)
    lat = oracle.Lattice(J, periodic, h)
    Es = energies(coupling_matrix(J, periodic), h, all_states(lat.n))
    betas = np.array([0.2, 0.45, 0.7, 0.95])
    slot_beta = np.tile(betas, 16)                        # 64 independent chains
    spins = oracle.apt_init(lat, 3, slot_beta.size, SEED)
    samples = [[] for _ in betas]
    t = 0
    for it in range(2000):
        oracle.apt_sweep(lat, 3, slot_beta, SEED, t, spins)
        t += 1
        if it >= 100 and it % 4 == 0:
            for s in range(slot_beta.size):
                samples[s % 4].append(oracle.energy(lat, spins[s]))
    for bi, beta in enumerate(betas):
        levels, p = boltzmann_energy_pmf(Es, beta)
        cnt = _energy_hist(levels, np.array(samples[bi]))
        pv, _, _ = chi2_pvalue(cnt, p)
        assert pv > 1e-4, (beta, pv)
        _, pwrong = boltzmann_energy_pmf(Es, beta * 1.25 + 0.05)
        assert chi2_pvalue(cnt, pwrong)[0] < 1e-6


def test_gibbs_full_state_distribution():
    """Every one of the 2^12 states of a 2x2x3 lattice (periodic z) at beta = 0.5."""
    J, _ = ej_couplings((2, 2, 3), 4, seed=12)
    lat = oracle.Lattice(J, 4)
    S = all_states(lat.n)
    Es = energies(coupling_matrix(J, 4), None, S)
    beta = 0.5
    w = np.exp(-beta * (Es - Es.min()))
    p = w / w.sum()
    codes = (((S + 1) // 2).astype(np.int64) << np.arange(lat.n)).sum(1)
    assert np.array_equal(codes, np.arange(S.shape[0]))
    spins = oracle.apt_init(lat, 0, 64, SEED)
    cnt = np.zeros(S.shape[0], np.int64)
    sb = np.full(64, beta)
    for it in range(1300):
        oracle.apt_sweep(lat, 0, sb, SEED, it, spins)
        if it >= 50 and it % 2 == 0:
            c = (((spins + 1) // 2).astype(np.int64) << np.arange(lat.n)).sum(1)
            np.add.at(cnt, c, 1)
    assert chi2_pvalue(cnt, p)[0] > 1e-4
    wb = np.exp(-0.7 * (Es - Es.min()))
    assert chi2_pvalue(cnt, wb / wb.sum())[0] < 1e-6


def test_sweep_result_independent_of_order_within_colour():
    """Sites of one colour are independent, so the sweep equals site-by-site Gibbs updates
    applied in any order inside each colour (here: descending), with the same random words."""
    J, _ = ej_couplings((5, 4, 3), 7, seed=13)
    lat = oracle.Lattice(J, 7)
    spins = oracle.apt_init(lat, 2, 8, SEED)
    ref = spins.copy()
    beta = np.linspace(0.3, 2.0, 8)
    oracle.apt_sweep(lat, 2, beta, SEED, 17, ref)
    for c in range(oracle.n_colours(lat)):
        for j in reversed(range(lat.n)):
            if oracle.colour(lat, j) != c:
                continue
            for s in range(8):
                I = oracle.local_field(lat, spins[s], j)
                u = oracle.word(SEED, j, 17, s >> 2, 2, oracle.TAG_APT_SWEEP, s & 3)
                spins[s, j] = 1 if u < oracle.heat_threshold(beta[s], I) else -1
    assert np.array_equal(spins, ref)


def test_replica_exchange_keeps_marginals_and_acceptance():
    J, _ = ej_couplings((2, 2, 3), 4, seed=14)
    lat = oracle.Lattice(J, 4)
    Es = energies(coupling_matrix(J, 4), None, all_states(lat.n))
    beta = np.array([0.3, 0.55, 0.9])
    R = 2
    spins = oracle.apt_init(lat, 1, beta.size * R, SEED)
    sb = np.repeat(beta, R)
    E = np.zeros(beta.size * R, np.int64)
    samples = [[] for _ in beta]
    trials = {}
    for cyc in range(6000):
        oracle.apt_sweep(lat, 1, sb, SEED, cyc, spins)
        for s in range(E.size):
            E[s] = oracle.energy(lat, spins[s])
        before = E.copy()
        acc = oracle.apt_swap(1, beta, R, SEED, cyc + 1, spins, E)
        for b in range(beta.size - 1):
            for l in range(R):
                a = acc[b * R + l]
                if a < 0:
                    continue
                dE = before[(b + 1) * R + l] - before[b * R + l]
                key = (b, int(dE))
                n_acc, n_tot = trials.get(key, (0, 0))
                trials[key] = (n_acc + a, n_tot + 1)
                if a:   # the exchanged states carry their energies
                    assert E[b * R + l] == before[(b + 1) * R + l]
        if cyc >= 200 and cyc % 2 == 0:
            for s in range(E.size):
                samples[s // R].append(E[s])
    for b, bt in enumerate(beta):
        levels, p = boltzmann_energy_pmf(Es, bt)
        cnt = _energy_hist(levels, np.array(samples[b]))
        assert chi2_pvalue(cnt, p)[0] > 1e-4
    checked = 0
    for (b, dE), (na, nt) in trials.items():
        pexp = min(1.0, math.exp((beta[b + 1] - beta[b]) * dE))
        if nt >= 200:
            checked += 1
            assert abs(na / nt - pexp) < 4.5 * math.sqrt(pexp * (1 - pexp) / nt) + 1e-9, (b, dE, na, nt)
    assert checked >= 6


def test_swap_pairs_alternate():
    """Odd attempts try (0,1),(2,3),...; even attempts (1,2),(3,4),... (Methods, APT details)."""
    beta = np.linspace(0.2, 1.5, 7)
    R = 2
    spins = np.ones((beta.size * R, 4), np.int8)
    E = np.arange(beta.size * R, dtype=np.int64)
    for a in (1, 2, 3, 4):
        acc = oracle.apt_swap(0, beta, R, SEED, a, spins.copy(), E.copy()).reshape(beta.size - 1, R)
        tried = acc[:, 0] >= 0
        assert np.array_equal(tried, np.arange(beta.size - 1) % 2 == (0 if a % 2 else 1))
        assert np.array_equal(acc[:, 0] >= 0, acc[:, 1] >= 0)


def _cluster_by_scipy(lat, A, B, seed_site):
    rows, cols = [], []
    for j in range(lat.n):
        for a in range(3):
            nb = oracle.neighbour(lat, j, a, 1)
            if nb >= 0 and oracle.bond(lat, j, a, 1) != 0 and A[j] != B[j] and A[nb] != B[nb]:
                rows.append(j); cols.append(nb)
    G = coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(lat.n, lat.n))
    _, lab = connected_components(G, directed=False)
    return set(np.flatnonzero(lab == lab[seed_site]).tolist())


@pytest.mark.parametrize("shape,periodic,R_lab,p_abs", [((6, 6, 6), 7, 2, 0.0), ((5, 4, 3), 3, 4, 0.0),
                                                        ((5, 5, 5), 7, 2, 0.3)])
def test_icm_invariants(shape, periodic, R_lab, p_abs):
    from paper_2503_10302_amd.inputs import diluted_couplings
    J = diluted_couplings(shape, periodic, seed=15, p_absent=p_abs)
    lat = oracle.Lattice(J, periodic)
    beta = np.array([0.4, 1.0, 1.3, 2.0])
    rng = np.random.default_rng(5)
    branches = set()
    for a in range(1, 25):
        spins = np.where(rng.random((beta.size * R_lab, lat.n)) < rng.random(), 1, -1).astype(np.int8)
        spins[R_lab:] = np.where(rng.random(spins[R_lab:].shape) < 0.2, -spins[R_lab:], spins[R_lab:])
        before = spins.copy()
        rc, info = oracle.apt_icm(lat, 4, beta, R_lab, 1.0, SEED, a, spins)
        assert rc == 0
        assert np.all(info[0] == -1) and np.array_equal(spins[:R_lab], before[:R_lab])   # below cutoff
        pairing = 0
        for b in range(1, beta.size):
            if R_lab == 4:
                w = oracle.word(SEED, b, a, 0, 4, oracle.TAG_ICM_PAIR, 0)
                pairing = (w * 3) >> 32
            pairs = [[(0, 1)], [(0, 1), (2, 3)], [(0, 2), (1, 3)], [(0, 3), (1, 2)]]
            plist = pairs[0] if R_lab == 2 else pairs[1 + pairing]
            for pi, (la, lb) in enumerate(plist):
                sa, sb = b * R_lab + la, b * R_lab + lb
                A0, B0, A1, B1 = before[sa], before[sb], spins[sa], spins[sb]
                m, seed_site, size, branch = (int(v) for v in info[b, pi])
                assert m == int(np.sum(A0 != B0))
                eA0, eB0 = oracle.energy(lat, A0), oracle.energy(lat, B0)
                assert oracle.energy(lat, A1) + oracle.energy(lat, B1) == eA0 + eB0   # isoenergetic
                if m == 0:
                    assert np.array_equal(A0, A1) and np.array_equal(B0, B1)
                    continue
                w0 = oracle.word(SEED, b * (R_lab // 2) + pi, a, 0, 4, oracle.TAG_ICM_PICK, 0)
                assert seed_site == np.flatnonzero(A0 != B0)[(w0 * m) >> 32]
                C = _cluster_by_scipy(lat, A0, B0, seed_site)
                assert size == len(C)
                branches.add(branch)
                if 2 * size > lat.n:
                    flipped = A1 if branch == 1 else B1
                    orig = A0 if branch == 1 else B0
                    assert np.array_equal(flipped, -orig)
                else:
                    assert branch == 0
                    assert set(np.flatnonzero(A0 != A1).tolist()) == C
                    assert set(np.flatnonzero(B0 != B1).tolist()) == C
                    assert np.array_equal(A1 * B1, A0 * B0)                        # overlap kept
    assert 0 in branches and (1 in branches or 2 in branches)


def test_icm_one_pair_per_call():
    """Four labels, one ICM per sweep (Supplementary comparison of one and two ICMs): at every
    temperature at or above the cutoff exactly one pair of the drawn matching is moved, each of
    the two with probability 1/2 (binomial, 5 sigma over 1200 temperature-calls), the other
    pair keeps its spins and gets the not-applied record, and the moved pair undergoes the
    same move as in the two-pair call (same record, same spins)."""
    J, _ = ej_couplings((5, 4, 4), 7, seed=19)
    lat = oracle.Lattice(J, 7)
    beta = np.array([0.4, 1.0, 1.3, 2.0, 2.5])
    rng = np.random.default_rng(6)
    first = 0
    total = 0
    for a in range(1, 301):
        spins = np.where(rng.random((beta.size * 4, lat.n)) < 0.5, 1, -1).astype(np.int8)
        both = spins.copy()
        rc, info = oracle.apt_icm(lat, 2, beta, 4, 1.0, SEED, a, spins, pairs_per_call=1)
        rc2, info2 = oracle.apt_icm(lat, 2, beta, 4, 1.0, SEED, a, both, pairs_per_call=2)
        assert rc == 0 and rc2 == 0 and np.all(info[0] == -1)
        for b in range(1, beta.size):
            applied = [pi for pi in range(2) if info[b, pi, 0] >= 0]
            assert len(applied) == 1, (a, b, info[b])
            pi = applied[0]
            first += pi == 0
            total += 1
            assert np.all(info[b, 1 - pi] == -1)
            assert np.array_equal(info[b, pi], info2[b, pi])
            w = oracle.word(SEED, b, a, 0, 2, oracle.TAG_ICM_PAIR, 0)
            pairing = (w * 3) >> 32
            plist = [[(0, 1), (2, 3)], [(0, 2), (1, 3)], [(0, 3), (1, 2)]][pairing]
            for lab in plist[pi]:
                assert np.array_equal(spins[b * 4 + lab], both[b * 4 + lab])
    assert abs(first - total / 2) <= 5 * 0.5 * np.sqrt(total), (first, total)


def test_icm_one_pair_leaves_the_other_pair_alone():
    J, _ = ej_couplings((4, 4, 4), 7, seed=20)
    lat = oracle.Lattice(J, 7)
    beta = np.array([1.2, 1.5, 2.0])
    rng = np.random.default_rng(7)
    for a in range(1, 60):
        spins = np.where(rng.random((beta.size * 4, lat.n)) < 0.5, 1, -1).astype(np.int8)
        before = spins.copy()
        _, info = oracle.apt_icm(lat, 0, beta, 4, 1.0, SEED, a, spins, pairs_per_call=1)
        for b in range(beta.size):
            pi = 0 if info[b, 0, 0] >= 0 else 1
            w = oracle.word(SEED, b, a, 0, 0, oracle.TAG_ICM_PAIR, 0)
            plist = [[(0, 1), (2, 3)], [(0, 2), (1, 3)], [(0, 3), (1, 2)]][(w * 3) >> 32]
            for lab in plist[1 - pi]:
                assert np.array_equal(spins[b * 4 + lab], before[b * 4 + lab])
            la, lb = plist[pi]
            E0 = oracle.energy(lat, before[b * 4 + la]) + oracle.energy(lat, before[b * 4 + lb])
            E1 = oracle.energy(lat, spins[b * 4 + la]) + oracle.energy(lat, spins[b * 4 + lb])
            assert E0 == E1


def test_icm_rejects_fields():
    J, h = ej_couplings((4, 4, 4), 7, seed=16, h_max=1)
    lat = oracle.Lattice(J, 7, h)
    spins = oracle.apt_init(lat, 0, 4, SEED)
    rc, _ = oracle.apt_icm(lat, 0, np.array([1.0, 2.0]), 2, 0.5, SEED, 1, spins)
    assert rc == -5
    before = spins.copy()
    rc, info = oracle.apt_icm(lat, 0, np.array([1.0, 2.0]), 2, 5.0, SEED, 1, spins)   # nothing applies
    assert rc == 0 and np.all(info == -1) and np.array_equal(spins, before)


def test_icm_with_gibbs_keeps_product_law():
    """Two replicas at the same beta with sweeps + ICM: each marginal stays Boltzmann."""
    J, _ = ej_couplings((2, 3, 3), 0, seed=17)
    lat = oracle.Lattice(J, 0)
    Es = energies(coupling_matrix(J, 0), None, all_states(lat.n))
    beta = np.array([0.8])
    spins = oracle.apt_init(lat, 0, 2, SEED)
    samples = []
    for cyc in range(12000):
        oracle.apt_sweep(lat, 0, np.full(2, 0.8), SEED, cyc, spins)
        oracle.apt_icm(lat, 0, beta, 2, 0.5, SEED, cyc + 1, spins)
        if cyc >= 100:
            samples += [oracle.energy(lat, spins[0]), oracle.energy(lat, spins[1])]
    levels, p = boltzmann_energy_pmf(Es, 0.8)
    cnt = _energy_hist(levels, np.array(samples))
    assert chi2_pvalue(cnt, p)[0] > 1e-4
    _, pw = boltzmann_energy_pmf(Es, 1.0)
    assert chi2_pvalue(cnt, pw)[0] < 1e-6


def test_apt_finds_brute_force_ground_state():
    J, _ = ej_couplings((2, 3, 3), 0, seed=18)
    lat = oracle.Lattice(J, 0)
    E0 = energies(coupling_matrix(J, 0), None, all_states(lat.n)).min()
    beta = np.geomspace(0.2, 3.0, 8)
    spins = oracle.apt_init(lat, 0, 16, SEED)
    counters = np.zeros(3, np.uint32)
    E = np.zeros(16, np.int64)
    best = np.array([np.iinfo(np.int64).max], np.int64)
    rc, trace, _ = oracle.apt_run(lat, 0, beta, 2, SEED, 300, 1, 1.0, 30, counters, spins, E, best)
    assert rc == 0 and best[0] == E0 and trace[-1] == E0
    assert np.all(np.diff(trace) <= 0) and counters.tolist() == [300, 300, 300]


def _sqa_exact(J, periodic, M, beta, gamma):
    """exp(-beta H_C) over all (n*M)-spin states; returns per-state (space, trotter) sums."""
    n = J.shape[0] * J.shape[1] * J.shape[2]
    W = coupling_matrix(J, periodic)
    S = all_states(n * M).reshape(-1, M, n).astype(np.float64)
    space = np.zeros(S.shape[0])
    for k in range(M):
        space += 0.5 * np.einsum("si,ij,sj->s", S[:, k], W, S[:, k])
    trot = np.zeros(S.shape[0])
    for k in range(M):
        trot += np.einsum("si,si->s", S[:, k], S[:, (k + 1) % M])
    K = -0.5 * math.log(math.tanh(beta * gamma / M))
    logw = (beta / M) * space + K * trot
    w = np.exp(logw - logw.max())
    return np.rint(space).astype(np.int64), np.rint(trot).astype(np.int64), w / w.sum()


@pytest.mark.parametrize("shape,periodic,M,gamma", [((2, 2, 1), 0, 4, 1.5), ((3, 2, 1), 1, 3, 0.8),
                                                    ((4, 1, 1), 1, 4, 2.5)])
def test_sqa_sweeps_sample_trotter_hamiltonian(shape, periodic, M, gamma):
    J, _ = ej_couplings(shape, periodic, seed=19)
    lat = oracle.Lattice(J, periodic)
    beta, R = 2.0, 32
    space, trot, p = _sqa_exact(J, periodic, M, beta, gamma)
    keys = space * 1000 + trot
    levels, inv = np.unique(keys, return_inverse=True)
    pk = np.bincount(inv, weights=p)
    spins = oracle.sqa_init(lat, 0, M, R, SEED)
    W = coupling_matrix(J, periodic)
    obs = []
    for t in range(1500):
        oracle.sqa_step(lat, 0, M, R, beta, gamma, SEED, t, spins)
        if t >= 100 and t % 3 == 0:
            sf = spins.astype(np.float64)
            sp = 0.5 * np.einsum("rki,ij,rkj->r", sf, W, sf)
            tr = np.einsum("rki,rki->r", sf, np.roll(sf, -1, axis=1))
            obs.append(np.rint(sp).astype(np.int64) * 1000 + np.rint(tr).astype(np.int64))
    obs = np.concatenate(obs)
    pos = np.searchsorted(levels, obs)
    assert np.all(levels[pos] == obs)
    cnt = np.bincount(pos, minlength=levels.size)
    assert chi2_pvalue(cnt, pk)[0] > 1e-4
    _, _, pw = _sqa_exact(J, periodic, M, beta, gamma * 1.4)
    assert chi2_pvalue(cnt, np.bincount(inv, weights=pw))[0] < 1e-6


def test_sqa_large_gamma_decouples_slices():
    """Gamma large: K -> 0 and every slice is an independent heat bath at beta / M."""
    J, _ = ej_couplings((2, 2, 3), 4, seed=20)
    lat = oracle.Lattice(J, 4)
    Es = energies(coupling_matrix(J, 4), None, all_states(lat.n))
    beta, M, R = 6.0, 4, 8
    spins = oracle.sqa_init(lat, 0, M, R, SEED)
    samples = []
    for t in range(900):
        oracle.sqa_step(lat, 0, M, R, beta, 500.0, SEED, t, spins)
        if t >= 50 and t % 2 == 0:
            samples += [oracle.energy(lat, s) for s in spins.reshape(-1, lat.n)]
    levels, p = boltzmann_energy_pmf(Es, beta / M)
    cnt = _energy_hist(levels, np.array(samples))
    assert chi2_pvalue(cnt, p)[0] > 1e-4
    assert chi2_pvalue(cnt, boltzmann_energy_pmf(Es, beta / M * 1.3)[1])[0] < 1e-6


def test_sqa_small_gamma_locks_slices():
    J, _ = ej_couplings((3, 3, 3), 7, seed=21)
    lat = oracle.Lattice(J, 7)
    M, R = 6, 2
    spins = oracle.sqa_init(lat, 0, M, R, SEED)
    spins[:] = spins[:, :1, :]                                  # every slice equal
    for t in range(50):
        oracle.sqa_step(lat, 0, M, R, 3.0, 1e-6, SEED, t, spins)
    assert np.all(spins == spins[:, :1, :])


def test_trotter_agreement_pins():
    """C_k from agreement counts: 1 at k = 0, -1 for a reversed slice, 0 within 5 sigma for the
    independent random slices of the initial state; after an anneal at vanishing transverse
    field (J_perp large) from a locked state every slice agrees with slice 0."""
    J, _ = ej_couplings((6, 5, 4), 7, seed=21)
    lat = oracle.Lattice(J, 7)
    M, R = 8, 6
    s = oracle.sqa_init(lat, 0, M, R, SEED)
    a = oracle.trotter_agreement(lat, s)
    assert np.all(a[:, 0] == lat.n)
    assert np.all(np.abs(a[:, 1:] - lat.n / 2) <= 5 * 0.5 * np.sqrt(lat.n))
    s2 = s.copy()
    s2[:, 3] = -s2[:, 0]
    assert np.all(oracle.trotter_agreement(lat, s2)[:, 3] == 0)
    locked = np.repeat(s[:, :1], M, axis=1).copy()
    oracle.sqa_anneal(lat, 0, M, R, 2.0, np.full(20, 1e-6), SEED, 0, locked)
    assert np.all(oracle.trotter_agreement(lat, locked) == lat.n)


def test_sqa_anneal_reports_minimum_slice():
    J, _ = ej_couplings((4, 4, 4), 7, seed=22)
    lat = oracle.Lattice(J, 7)
    M, R = 4, 3
    spins = oracle.sqa_init(lat, 0, M, R, SEED)
    g = np.linspace(3.0, 0.01, 30)
    bE, bs, sE = oracle.sqa_anneal(lat, 0, M, R, 2.0, g, SEED, 0, spins)
    flat = spins.reshape(-1, lat.n)
    assert bE == sE.min() == oracle.energy(lat, bs)
    assert np.array_equal(bs, flat[int(np.argmin(sE.reshape(-1)))])
    assert all(sE.reshape(-1)[q] == oracle.energy(lat, flat[q]) for q in range(M * R))


def test_adaptive_ladder_independent_spins_closed_form():
    """No couplings, h = 1: E = -sum s, sigma_E(beta) = sqrt(n) sech(beta) exactly."""
    J = np.zeros((4, 4, 4, 3), np.int8)
    h = np.ones(64, np.int8)
    lat = oracle.Lattice(J, 7, h)
    betas, sig, mom = oracle.adaptive_ladder(lat, 0, SEED, beta0=0.5, alpha=1.25, tol=0.5,
                                             n_chains=20, sweeps=600, tail=500, max_steps=30)
    assert betas[0] == 0.5
    for b, s in zip(betas, sig):
        exact = 8.0 / math.cosh(b)
        if exact >= 1.0:     # rare-flip regime: the mean sample std is biased low
            assert abs(s - exact) < 0.035 * exact
        else:
            assert abs(s - exact) < 0.15 * exact
    for t in range(len(betas) - 1):
        assert betas[t + 1] == betas[t] + 1.25 / sig[t]
        assert sig[t] >= 0.5
    assert sig[-1] < 0.5
    # sigma_E is the mean of per-chain sample standard deviations from integer moments
    for t in range(len(betas)):
        per = [oracle.sigma_from_moments(m[0], m[1], 500) for m in mom[t]]
        assert sig[t] == sum(per) / len(per)


def test_sigma_from_moments_matches_sample_std():
    rng = np.random.default_rng(9)
    x = rng.integers(-500, 500, size=777)
    assert abs(oracle.sigma_from_moments(x.sum(), (x * x).sum(), x.size) - x.std(ddof=1)) < 1e-9 * x.std()


def test_adaptive_ladder_gives_erfc_acceptance():
    """Near-Gaussian energies with dbeta * sigma_E = alpha: acceptance ~ erfc(alpha/2) = 0.377."""
    J = np.zeros((6, 6, 6, 3), np.int8)
    h = np.ones(216, np.int8)
    lat = oracle.Lattice(J, 7, h)
    betas, sig, _ = oracle.adaptive_ladder(lat, 0, SEED, beta0=0.3, alpha=1.25, tol=3.0,
                                           n_chains=8, sweeps=300, tail=250, max_steps=6)
    assert len(betas) >= 4
    R = 1
    spins = oracle.apt_init(lat, 0, betas.size, SEED)
    E = np.zeros(betas.size, np.int64)
    acc_n = np.zeros(betas.size - 1)
    tot_n = np.zeros(betas.size - 1)
    for cyc in range(3000):
        oracle.apt_sweep(lat, 0, betas, SEED, cyc, spins)
        for s in range(betas.size):
            E[s] = oracle.energy(lat, spins[s])
        acc = oracle.apt_swap(0, betas, R, SEED, cyc + 1, spins, E)
        acc_n += np.maximum(acc, 0)
        tot_n += acc >= 0
    rate = acc_n / tot_n
    assert np.all(np.abs(rate - erfc(1.25 / 2)) < 0.06), rate


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(10)
    P = rng.normal(0, 0.3, oracle.MLP_NPARAM)
    x = rng.normal(0, 1, (5, 4))
    y = rng.normal(0, 1, (5, 33))
    loss, g, out = oracle.mlp_loss_grad(P, x, y)
    assert np.all(np.diff(out[:, :32], axis=1) > 0)          # monotone ladder
    idx = rng.choice(P.size, 60, replace=False)
    eps = 1e-6
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += eps; Pm[i] -= eps
        fd = (oracle.mlp_loss_grad(Pp, x, y)[0] - oracle.mlp_loss_grad(Pm, x, y)[0]) / (2 * eps)
        assert abs(fd - g[i]) < 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_instance_features():
    J, _ = ej_couplings((4, 4, 4), 7, seed=23)
    f = oracle.instance_features(oracle.Lattice(J, 7))
    assert abs(f[0] - 4.0) < 1e-12
    sums = np.zeros((4, 4, 4))
    for a in range(3):
        sums += J[..., a] + np.roll(J[..., a], 1, axis=2 - a)
    v = np.abs(sums).ravel()
    assert abs(f[1] - v.mean()) < 1e-12 and abs(f[2] - v.var()) < 1e-12
    frus = tot = 0
    for a in range(3):
        for b in range(a + 1, 3):
            p = (J[..., a] * np.roll(J[..., b], -1, axis=2 - a) * np.roll(J[..., a], -1, axis=2 - b)
                 * J[..., b])
            frus += int((p < 0).sum()); tot += p.size
    assert abs(f[3] - frus / tot) < 1e-12
    ferro = np.ones((4, 4, 4, 3), np.int8)
    assert oracle.instance_features(oracle.Lattice(ferro, 7))[3] == 0.0
