"""Host-side pieces of the learned-ladder module (no GPU): ladder resampling, the cutoff
label, network targets, the per-pair acceptance bookkeeping and the band check."""
import math

import numpy as np

import oracle
from paper_2503_10302_amd import ladder


def test_resample_keeps_endpoints_order_and_identity():
    rng = np.random.default_rng(3)
    b = np.cumsum(rng.uniform(0.01, 0.3, 20)) + 0.5
    r = ladder.resample(b)
    assert r.size == ladder.N_RUNGS
    assert r[0] == b[0] and r[-1] == b[-1]
    assert np.all(np.diff(r) > 0)
    b32 = np.cumsum(rng.uniform(0.01, 0.3, 32)) + 0.5
    np.testing.assert_array_equal(ladder.resample(b32), b32)
    # a linear ladder stays linear
    np.testing.assert_allclose(ladder.resample(np.linspace(0.5, 3.0, 7)), np.linspace(0.5, 3.0, 32))


def test_cutoff_label_is_first_rung_at_or_above_one():
    assert ladder.cutoff_label([0.5, 0.9, 1.0, 1.2]) == 1.0
    assert ladder.cutoff_label([0.5, 0.9, 1.1, 1.2]) == 1.1
    assert ladder.cutoff_label([0.5, 0.7, 0.9]) == 0.9


def test_targets_are_log_ladder_and_log_cutoff():
    b = np.array([0.5, 0.6, 0.8, 1.05, 1.5, 2.5])
    t = ladder.targets(b)
    assert t.shape == (ladder.N_RUNGS + 1,)
    np.testing.assert_allclose(np.exp(t[:ladder.N_RUNGS]), ladder.resample(b), rtol=1e-14)
    assert math.isclose(math.exp(t[-1]), ladder.cutoff_label(ladder.resample(b)), rel_tol=1e-14)


def test_attempt_counts_follow_the_swap_schedule():
    """acceptance() divides by the number of attempts each pair had; count the attempts the
    oracle's swap step actually makes (a flag other than -1) and check that counting every
    attempt as accepted gives exactly 1 for every pair."""
    n_beta, R, n = 6, 2, 8
    beta = np.linspace(0.5, 1.5, n_beta)
    spins = np.ones((n_beta * R, n), np.int8)
    E = np.zeros(n_beta * R, np.int64)
    for cycles in (1, 2, 7, 10):
        attempted = np.zeros((n_beta - 1) * R, np.int64)
        for a in range(1, cycles + 1):
            flags = oracle.apt_swap(0, beta, R, 99, a, spins, E)
            attempted += flags != -1
        acc = ladder.acceptance(attempted[None, :], cycles, n_beta, R)
        if cycles == 1:     # only the even pairs have been tried
            np.testing.assert_array_equal(acc[0, 0::2], 1.0)
            assert np.isnan(acc[0, 1::2]).all()
            assert not ladder.in_band(acc)[0]
        else:
            np.testing.assert_array_equal(acc, np.ones((1, n_beta - 1)))


def test_band_checks_every_pair():
    """The default band [0.5, 1.5] x erfc(alpha / 2) on every adjacent pair, and per-pair bands
    (arrays) as the calibrated tables give them: a cold pair below its own bound fails, above it
    passes."""
    lo, hi = ladder.BAND
    assert math.isclose(lo, 0.5 * math.erfc(1.25 / 2)) and math.isclose(hi, 1.5 * math.erfc(1.25 / 2))
    good = np.full((1, 31), 0.38)
    cold = good.copy()
    cold[0, -2:] = [0.1, 0.02]
    warm = good.copy()
    warm[0, 3] = 0.1
    high = good.copy()
    high[0, 0] = 0.9
    acc = np.concatenate([good, cold, warm, high])
    np.testing.assert_array_equal(ladder.in_band(acc), [True, False, False, False])
    plo = np.full(31, lo)
    phi = np.full(31, hi)
    plo[-2:] = [0.05, 0.01]
    np.testing.assert_array_equal(ladder.in_band(acc, plo, phi), [True, True, False, False])
    plo[-1] = 0.03
    np.testing.assert_array_equal(ladder.in_band(acc, plo, phi), [True, False, False, False])


def test_tables_by_nearest_size():
    """Per-size tables are looked up by the size nearest to each instance's cube root of n;
    without tables every instance gets the default band."""
    from paper_2503_10302_amd.inputs import ej_couplings
    t = {"sizes": np.array([8, 10, 12, 15]), "band_lo": np.arange(4)[:, None] * np.ones((4, 31)),
         "band_hi": 10 + np.arange(4)[:, None] * np.ones((4, 31)),
         "size_mean": np.log(np.arange(1, 5))[:, None] * np.ones((4, 33))}
    inst = [(ej_couplings(L, 7, seed=1)[0], 7, None) for L in (8, 9, 11, 15, 6)]
    lo, hi = ladder.bands_for(inst, t)
    np.testing.assert_array_equal(lo[:, 0], [0, 0, 1, 3, 0])   # 9 -> 8 (tie to the first), 11 -> 10
    np.testing.assert_array_equal(hi[:, 5], [10, 10, 11, 13, 10])
    b, c = ladder.table_ladders(inst, t)
    np.testing.assert_allclose(b[:, 0], [1, 1, 2, 4, 1])
    lo0, hi0 = ladder.bands_for(inst, None)
    assert np.all(lo0 == ladder.BAND[0]) and np.all(hi0 == ladder.BAND[1])


def test_dilution_is_per_instance_and_reproducible():
    d = [ladder.dilution_of(i, 30000, 0.3) for i in range(200)]
    assert d == [ladder.dilution_of(i, 30000, 0.3) for i in range(200)]
    assert 0 <= min(d) and max(d) < 0.3 and np.std(d) > 0.07
    assert ladder.dilution_of(5, 30000, 0.0) == 0.0


def _geom(n=32, lo=0.4, hi=3.2):
    return lo * (hi / lo) ** (np.arange(n) / (n - 1))


def test_repair_keeps_a_ladder_whose_pairs_sit_at_the_band_middle():
    """Acceptances exactly at the middle of every pair's band: the measured and wanted lengths
    coincide and the repair returns the ladder itself (to rounding)."""
    rng = np.random.default_rng(5)
    b = _geom()
    mid = rng.uniform(0.1, 0.5, 31)
    lo, hi = mid - 0.05, mid + 0.05
    out = ladder.repair(b, 0.5 * (lo + hi), lo, hi)
    np.testing.assert_allclose(out, b, rtol=1e-12)
    assert out[0] == b[0] and out[-1] == b[-1]


def test_repair_gives_every_pair_its_wanted_length_under_the_gaussian_model():
    """Model check: an instance whose pair lengths (dbeta sigma) are x_b has pilot acceptance
    erfc(x_b / 2); with the length taken as linear in log beta between the old rungs, the
    repaired rungs must cut the instance's total length in the proportions of the band
    midpoints' lengths 2 erfc^-1(m_b).  When the totals agree, each repaired pair has exactly
    its wanted length, i.e. acceptance m_b under the model.  The lengths of the repaired
    pairs are measured here with numpy interpolation, independently of the library."""
    from scipy import special
    rng = np.random.default_rng(11)
    b = _geom()
    x = rng.uniform(0.4, 3.5, 31)              # measured pair lengths, some far off
    acc = special.erfc(x / 2)
    y = rng.uniform(0.8, 2.2, 31)
    y *= x.sum() / y.sum()                     # wanted lengths with the same total
    mid = special.erfc(y / 2)
    lo, hi = mid - 0.02, mid + 0.02
    out = ladder.repair(b, acc, lo, hi)
    S = np.concatenate([[0.0], np.cumsum(x)])
    s_new = np.interp(np.log(out), np.log(b), S)
    np.testing.assert_allclose(np.diff(s_new), y, rtol=0, atol=1e-9)
    np.testing.assert_allclose(special.erfc(np.diff(s_new) / 2), mid, atol=1e-9)
    # totals that disagree: lengths scale by one common factor, ends fixed
    out2 = ladder.repair(b, special.erfc(1.3 * x / 2), lo, hi)
    s2 = np.interp(np.log(out2), np.log(b), 1.3 * S)
    np.testing.assert_allclose(np.diff(s2), 1.3 * y, atol=1e-9)


def test_repair_damping_is_a_geometric_mix():
    """Damping d gives exp((1 - d) log beta + d log beta_full) rung by rung."""
    rng = np.random.default_rng(2)
    b = _geom()
    acc = rng.uniform(0.05, 0.7, 31)
    lo, hi = np.full(31, 0.2), np.full(31, 0.5)
    full = ladder.repair(b, acc, lo, hi, 1.0)
    half = ladder.repair(b, acc, lo, hi, 0.5)
    np.testing.assert_allclose(half, np.sqrt(b * full), rtol=1e-12)
    q = ladder.repair(b, acc, lo, hi, 0.25)
    np.testing.assert_allclose(q, np.exp(0.75 * np.log(b) + 0.25 * np.log(full)), rtol=1e-12)


def test_repair_extremes_and_errors():
    """Acceptances of 0 and 1 (clamped) still give a strictly ascending ladder with the same
    ends; invalid arguments are refused."""
    from paper_2503_10302_amd import sg
    b = _geom()
    acc = np.tile([0.0, 1.0, 0.3], 11)[:31]
    out = ladder.repair(b, acc, np.full(31, 0.2), np.full(31, 0.5))
    assert out[0] == b[0] and out[-1] == b[-1] and np.all(np.diff(out) > 0)
    lo, hi = np.full(31, 0.2), np.full(31, 0.5)
    bad = [(b[::-1], np.full(31, 0.3), lo, hi, 1.0),          # descending
           (b, np.full(31, 1.5), lo, hi, 1.0),                # acceptance > 1
           (b, np.full(31, 0.3), hi, lo, 1.0),                # empty band
           (b, np.full(31, 0.3), lo, hi, 0.0),                # damping 0
           (b, np.full(31, 0.3), lo, hi, 1.5)]                # damping > 1
    for args in bad:
        try:
            ladder.repair(*args[:4], damping=args[4])
        except sg.SGError as e:
            assert e.code == sg.SG_EINVAL
        else:
            raise AssertionError("accepted invalid arguments")


def test_mean_rho_crossing_averages_over_instances():
    """Eq. (2): the residual energy per spin is averaged over the instances before the target
    is applied, so one slow instance delays the crossing only by its share of the mean."""
    E0 = np.array([-100, -200])
    n = np.array([10, 20])
    # instance 0 reaches E0 at cycle 3; instance 1 stays 2 above E0 (rho 0.1) throughout
    tr = np.array([[-90, -95, -100, -100, -100],
                   [-198, -198, -198, -198, -198]])
    # mean rho per cycle: (1.0 + 0.1)/2, (0.5 + 0.1)/2, (0 + 0.1)/2, ...
    assert ladder.mean_rho_cycles(tr, E0, n, 0.05) == 3
    assert ladder.mean_rho_cycles(tr, E0, n, 0.3) == 2
    assert ladder.mean_rho_cycles(tr, E0, n, 0.01) == -1
