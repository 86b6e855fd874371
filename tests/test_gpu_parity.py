"""GPU parity: libsg (HIP, through the C ABI) against the CPU oracle, bit for bit.

Spins, energies, ICM records, swap decisions, running minima, DT-SQA slice
energies and adaptive ladders must be identical: every decision on both sides
is an integer comparison of the same Philox word with the same FP64-built
threshold.  Sizes span several work-group tiles, ragged site counts (n not a
multiple of 4 or 16), three-colour lattices (odd periodic axes), open axes,
missing bonds and fields.  Full-size workloads are checked on sampled
instances / replicas that the oracle recomputes one at a time.
"""
import numpy as np
import pytest

import oracle
from paper_2503_10302_amd import sg
from paper_2503_10302_amd.inputs import (diluted_couplings, ej_couplings, geometric_ladder,
                                         linear_gamma, missing_spin_couplings, mixed_sizes)

pytestmark = pytest.mark.gpu
SEED = 0x5EED_1234_ABCD


def _inst(shape, periodic, seed, hmax=0, p_absent=0.0):
    if p_absent > 0:
        return (diluted_couplings(shape, periodic, seed, p_absent), periodic, None)
    J, h = ej_couplings(shape, periodic, seed, h_max=hmax)
    return (J, periodic, h)


def _olat(inst):
    return oracle.Lattice(inst[0], inst[1], inst[2])


def _gpu_slots(ctx, i, n):
    return ctx.spins()[i, :, :n]


MIXED = [((5, 5, 5), 7, 1, 0, 0.0), ((4, 4, 4), 7, 2, 0, 0.0), ((6, 3, 4), 5, 3, 0, 0.0),
         ((7, 6, 5), 7, 4, 0, 0.0), ((6, 6, 6), 7, 5, 0, 0.25), ((3, 5, 2), 0, 6, 0, 0.0),
         ((9, 9, 9), 7, 7, 0, 0.0), ((2, 2, 2), 7, 8, 0, 0.0)]


@pytest.mark.parametrize("reps", [2, 4, 1])
def test_apt_calls_match_oracle(reps):
    insts = [_inst(*m) for m in MIXED]
    beta = geometric_ladder(8, 0.2, 3.0)
    ctx = sg.apt(insts, beta, SEED, reps_per_beta=reps)
    lats = [_olat(x) for x in insts]
    ns = [l.n for l in lats]
    nslot = beta.size * reps
    sb = np.repeat(beta, reps)
    ospins = [oracle.apt_init(l, i, nslot, SEED) for i, l in enumerate(lats)]
    g = ctx.spins()
    for i in range(len(insts)):
        assert np.array_equal(g[i, :, :ns[i]], ospins[i]), f"init, instance {i}"
    E0 = ctx.energy()
    for i, l in enumerate(lats):
        assert [oracle.energy(l, s) for s in ospins[i]] == E0[i].tolist()
    t = 0
    for cyc in range(3):
        ctx.sweep(2)
        for i, l in enumerate(lats):
            for k in range(2):
                oracle.apt_sweep(l, i, sb, SEED, t + k, ospins[i])
        t += 2
        g = ctx.spins()
        E = ctx.energy()
        for i, l in enumerate(lats):
            assert np.array_equal(g[i, :, :ns[i]], ospins[i]), f"sweep cycle {cyc} instance {i}"
            assert E[i].tolist() == [oracle.energy(l, s) for s in ospins[i]]
        if reps >= 2:
            info = ctx.icm(0.8, want_info=True)
            for i, l in enumerate(lats):
                rc, oinfo = oracle.apt_icm(l, i, beta, reps, 0.8, SEED, cyc + 1, ospins[i])
                assert rc == 0
                assert np.array_equal(info[i], oinfo), f"icm records, instance {i}"
            g = ctx.spins()
            for i in range(len(lats)):
                assert np.array_equal(g[i, :, :ns[i]], ospins[i]), f"icm cycle {cyc} instance {i}"
        E = ctx.energy()
        acc = ctx.swap()
        for i, l in enumerate(lats):
            Eo = np.array([oracle.energy(l, s) for s in ospins[i]], np.int64)
            assert np.array_equal(E[i], Eo)
            oacc = oracle.apt_swap(i, beta, reps, SEED, cyc + 1, ospins[i], Eo)
            assert np.array_equal(acc[i], oacc), f"swap flags, instance {i}"
        g = ctx.spins()
        for i in range(len(lats)):
            assert np.array_equal(g[i, :, :ns[i]], ospins[i]), f"after swap {cyc}, instance {i}"
    assert ctx.counters().tolist() == [t, 3 if reps >= 2 else 0, 3]


@pytest.mark.parametrize("reps,S,cutoff", [(2, 1, 1.0), (4, 2, 0.5), (2, 3, float("inf")), (1, 1, 1.0)])
def test_apt_cycles_match_oracle(reps, S, cutoff):
    insts = [_inst(*m) for m in MIXED[:6]]
    beta = geometric_ladder(10, 0.2, 3.0)
    ctx = sg.apt(insts, beta, SEED + reps, reps_per_beta=reps)
    n_cyc = 77                                   # two replays of the 32-cycle graph plus a ragged tail
    trace = ctx.run_apt(n_cyc, S, cutoff, record_every=5)
    g = ctx.spins()
    best = ctx.best()
    cnt = ctx.swap_counts()
    for i, inst in enumerate(insts):
        l = _olat(inst)
        sp = oracle.apt_init(l, i, beta.size * reps, SEED + reps)
        ctr = np.zeros(3, np.uint32)
        E = np.zeros(beta.size * reps, np.int64)
        b = np.array([np.iinfo(np.int64).max], np.int64)
        rc, otr, oacc = oracle.apt_run(l, i, beta, reps, SEED + reps, n_cyc, S, cutoff, 5, ctr, sp, E, b)
        assert rc == 0
        assert np.array_equal(g[i, :, :l.n], sp), f"instance {i}"
        assert np.array_equal(trace[i], otr)
        assert best[i] == b[0]
        assert np.array_equal(cnt[i], oacc)
    assert ctx.counters().tolist() == [n_cyc * S, n_cyc, n_cyc]


@pytest.mark.parametrize("code", [0, 14])
@pytest.mark.parametrize("reps,pairs,S", [(4, 1, 1), (4, 2, 10), (2, 1, 1)])
def test_apt_options_match_oracle(reps, pairs, S, code):
    """sg_run_apt_ex: one or two Houdayer moves per temperature per cycle (four labels), a
    sweep-to-swap ratio of 10, and a different ICM cutoff per instance, against the oracle
    (each instance run with its own cutoff): spins, best-energy traces, swap counts, over two
    replays of the 32-cycle graph and a ragged tail; with the autotuner's launch configuration
    and with two launch groups on two streams (code 14)."""
    insts = [_inst(*m) for m in MIXED[:6]]
    beta = geometric_ladder(10, 0.2, 3.0)
    cut = np.array([0.2, 1.0, 0.6, float("inf"), 1.5, 0.9])
    ctx = sg.apt(insts, beta, SEED + 7 * reps + pairs, reps_per_beta=reps)
    if code:
        ctx.set_launch_config(code)
    n_cyc = 70
    trace = ctx.run_apt_ex(n_cyc, S, cut, pairs, record_every=7)
    g = ctx.spins()
    cnt = ctx.swap_counts()
    for i, inst in enumerate(insts):
        l = _olat(inst)
        sp = oracle.apt_init(l, i, beta.size * reps, SEED + 7 * reps + pairs)
        ctr = np.zeros(3, np.uint32)
        E = np.zeros(beta.size * reps, np.int64)
        b = np.array([np.iinfo(np.int64).max], np.int64)
        rc, otr, oacc = oracle.apt_run(l, i, beta, reps, SEED + 7 * reps + pairs, n_cyc, S, cut[i], 7,
                                       ctr, sp, E, b, icm_pairs=pairs)
        assert rc == 0
        assert np.array_equal(g[i, :, :l.n], sp), f"instance {i}"
        assert np.array_equal(trace[i], otr), f"trace, instance {i}"
        assert np.array_equal(cnt[i], oacc)


def test_apt_sweep_to_swap_ratio_516_matches_oracle():
    """The ablation's largest sweep-to-swap ratio: 516 sweeps in each cycle's launch (the
    packed energy sums flushed every sweep), then the cluster moves and the exchange, over
    three cycles and two labels, against the oracle."""
    insts = [_inst((5, 4, 3), 7, 97), _inst((4, 4, 4), 7, 98)]
    beta = geometric_ladder(6, 0.3, 2.5)
    ctx = sg.apt(insts, beta, SEED + 516, reps_per_beta=2)
    trace = ctx.run_apt(3, 516, 1.0, record_every=1)
    g = ctx.spins()
    E = ctx.energy()
    for i, inst in enumerate(insts):
        l = _olat(inst)
        sp = oracle.apt_init(l, i, 12, SEED + 516)
        ctr = np.zeros(3, np.uint32)
        Eo = np.zeros(12, np.int64)
        b = np.array([np.iinfo(np.int64).max], np.int64)
        rc, otr, _ = oracle.apt_run(l, i, beta, 2, SEED + 516, 3, 516, 1.0, 1, ctr, sp, Eo, b)
        assert rc == 0 and np.array_equal(g[i, :, :l.n], sp), f"instance {i}"
        assert np.array_equal(trace[i], otr), f"instance {i}"
        assert E[i].tolist() == [oracle.energy(l, s_) for s_ in sp], f"instance {i}"


def test_apt_every_launch_config_matches_oracle():
    """Every APT launch configuration (six work-group orders x 7 or 8 waves per SIMD, and the
    three splits into two launch groups on two streams) gives the oracle's spins, traces and
    swap counts, over a 32-cycle graph replay and a tail."""
    insts = [_inst(*m) for m in MIXED]
    beta = geometric_ladder(8, 0.2, 3.0)
    ref = []
    for i, inst in enumerate(insts):
        l = _olat(inst)
        sp = oracle.apt_init(l, i, beta.size * 2, SEED + 5)
        ctr = np.zeros(3, np.uint32)
        E = np.zeros(beta.size * 2, np.int64)
        b = np.array([np.iinfo(np.int64).max], np.int64)
        rc, otr, oacc = oracle.apt_run(l, i, beta, 2, SEED + 5, 37, 1, 1.0, 1, ctr, sp, E, b)
        assert rc == 0
        ref.append((l.n, sp, otr, oacc))
    for code in range(1, 16):
        ctx = sg.apt(insts, beta, SEED + 5, reps_per_beta=2)
        ctx.set_launch_config(code)
        assert ctx.launch_config() == code
        tr = ctx.run_apt(37, 1, 1.0, record_every=1)
        g = ctx.spins()
        cnt = ctx.swap_counts()
        for i, (n, sp, otr, oacc) in enumerate(ref):
            assert np.array_equal(g[i, :, :n], sp), f"config {code}, instance {i}"
            assert np.array_equal(tr[i], otr) and np.array_equal(cnt[i], oacc), f"config {code}"
        ctx.close()
    # a split that leaves the second group empty (one instance) runs as one group
    one = sg.apt(insts[6:7], beta, SEED + 5, reps_per_beta=2)
    one.set_launch_config(14)
    tr = one.run_apt(37, 1, 1.0, record_every=1)
    l6 = _olat(insts[6])
    sp = oracle.apt_init(l6, 0, beta.size * 2, SEED + 5)
    ctr = np.zeros(3, np.uint32)
    E = np.zeros(beta.size * 2, np.int64)
    b = np.array([np.iinfo(np.int64).max], np.int64)
    rc, otr, _ = oracle.apt_run(l6, 0, beta, 2, SEED + 5, 37, 1, 1.0, 1, ctr, sp, E, b)
    assert rc == 0 and np.array_equal(one.spins()[0, :, :l6.n], sp) and np.array_equal(tr[0], otr)
    one.close()
    ctx = sg.apt(insts, beta, SEED + 5, reps_per_beta=2)
    for bad in (-1, 16, 1000):
        with pytest.raises(sg.SGError) as e:
            ctx.set_launch_config(bad)
        assert e.value.code == sg.SG_EINVAL


def test_apt_autotuner_keeps_state_and_caches(tmp_path, monkeypatch):
    """The first run of a context with no configuration times the fifteen candidates on a saved
    copy of the state and restores it: the run still matches the oracle; the pick is kept by
    the context, in the process cache and in the on-disk cache file."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("SG_TUNE_CACHE", str(cache))
    insts = [_inst(*m) for m in MIXED[:5]] + [_inst((11, 10, 9), 7, 44)]
    beta = geometric_ladder(12, 0.2, 3.0)
    ctx = sg.apt(insts, beta, SEED + 6, reps_per_beta=4)
    assert ctx.launch_config() == 0
    ctx.sweep(3)
    tr = ctx.run_apt_ex(45, 1, 0.9, 1, record_every=3)
    code = ctx.launch_config()
    assert 1 <= code <= 15
    g = ctx.spins()
    for i, inst in enumerate(insts):
        l = _olat(inst)
        sp = oracle.apt_init(l, i, beta.size * 4, SEED + 6)
        for t in range(3):
            oracle.apt_sweep(l, i, np.repeat(beta, 4), SEED + 6, t, sp)
        ctr = np.array([3, 0, 0], np.uint32)
        E = np.array([oracle.energy(l, x) for x in sp], np.int64)
        b = np.array([np.iinfo(np.int64).max], np.int64)
        rc, otr, _ = oracle.apt_run(l, i, beta, 4, SEED + 6, 45, 1, 0.9, 3, ctr, sp, E, b, icm_pairs=1)
        assert rc == 0
        assert np.array_equal(g[i, :, :l.n], sp), f"instance {i}"
        assert np.array_equal(tr[i], otr)
    lines = cache.read_text().split("\n")
    assert any(l.endswith(f" {code}") for l in lines if l)
    again = sg.apt(insts, beta, SEED + 7, reps_per_beta=4)
    again.run_apt_ex(2, 1, 0.9, 1)
    assert again.launch_config() == code


def test_icm_one_pair_records_match_oracle():
    """sg_icm_ex with one move per temperature: the (m, seed, |C|, branch) record of the moved
    pair and the not-applied record of the other, per temperature, equal the oracle's."""
    insts = [_inst(*m) for m in MIXED]
    beta = geometric_ladder(8, 0.2, 3.0)
    ctx = sg.apt(insts, beta, SEED + 99, reps_per_beta=4)
    lats = [_olat(x) for x in insts]
    osp = [oracle.apt_init(l, i, beta.size * 4, SEED + 99) for i, l in enumerate(lats)]
    cut = np.array([0.5, 1.0, 0.2, 2.0, 0.7, 0.3, 1.1, 0.9])
    for call in range(1, 4):
        ctx.sweep(1)
        for i, l in enumerate(lats):
            oracle.apt_sweep(l, i, np.repeat(beta, 4), SEED + 99, call - 1, osp[i])
        info = ctx.icm_ex(cut, icm_pairs=1, want_info=True)
        g = ctx.spins()
        for i, l in enumerate(lats):
            rc, oinfo = oracle.apt_icm(l, i, beta, 4, cut[i], SEED + 99, call, osp[i], pairs_per_call=1)
            assert rc == 0
            assert np.array_equal(info[i], oinfo), f"call {call}, instance {i}"
            assert np.array_equal(g[i, :, :l.n], osp[i]), f"call {call}, instance {i}"


def _coloured_instances():
    """Irregular instances with given colour maps: DSATUR maps of a heavily diluted odd
    periodic lattice, a lattice with a missing spin (open x, y) and an odd periodic cube, and a
    four-colour map (checkerboard classes split at random) of an even periodic cube."""
    insts = [(diluted_couplings((7, 6, 5), 7, 31, 0.75), 7, None),
             (missing_spin_couplings((10, 10, 10), 4, 32, 1), 4, None),
             (ej_couplings((5, 5, 5), 7, 33)[0], 7, None),
             (ej_couplings((6, 6, 4), 7, 34)[0], 7, None)]
    maps = [sg.dsatur(x)[0] for x in insts[:3]]
    base = (np.indices((4, 6, 6)).sum(axis=0) % 2).reshape(-1)
    maps.append((base + 2 * (np.random.default_rng(35).random(base.size) < 0.5)).astype(np.int8))
    return insts, maps


def test_colour_maps_apt_match_oracle():
    """APT+ICM with given colour maps against the oracle with the same maps: spins, traces and
    swap counts.  The maps include two colours on an odd lattice (dilution removed its odd
    cycles; the closed form would use three) and four colours."""
    insts, maps = _coloured_instances()
    ncol = [int(m.max()) + 1 for m in maps]
    assert 4 in ncol and ncol[0] == 2
    beta = geometric_ladder(8, 0.2, 3.0)
    ctx = sg.apt(insts, beta, SEED + 11, reps_per_beta=2, colours=maps)
    tr = ctx.run_apt(40, 1, 1.0, record_every=4)
    g = ctx.spins()
    for i, ((J, per, h), m) in enumerate(zip(insts, maps)):
        l = oracle.Lattice(J, per, h, m)
        sp = oracle.apt_init(l, i, beta.size * 2, SEED + 11)
        ctr = np.zeros(3, np.uint32)
        E = np.zeros(beta.size * 2, np.int64)
        b = np.array([np.iinfo(np.int64).max], np.int64)
        rc, otr, _ = oracle.apt_run(l, i, beta, 2, SEED + 11, 40, 1, 1.0, 4, ctr, sp, E, b)
        assert rc == 0
        assert np.array_equal(g[i, :, :l.n], sp), f"instance {i}"
        assert np.array_equal(tr[i], otr), f"instance {i}"


@pytest.mark.parametrize("M", [8, 7])
def test_colour_maps_sqa_match_oracle(M):
    """DT-SQA with the same maps (slice k of site j coloured (map[j] + t(k)) mod C, t(k) = k mod 2
    but t(M - 1) = 2 for odd M): spins, slice energies and the minimum, against the oracle."""
    insts, maps = _coloured_instances()
    R, beta = 3, 2.0
    ctx = sg.sqa(insts, M, R, beta, SEED + 12, colours=maps)
    gam = linear_gamma(9)
    bE, bs = ctx.sqa_anneal(gam)
    g = ctx.spins()
    E = ctx.energy()
    for i, ((J, per, h), m) in enumerate(zip(insts, maps)):
        l = oracle.Lattice(J, per, h, m)
        sp = oracle.sqa_init(l, i, M, R, SEED + 12)
        obE, obs, osE = oracle.sqa_anneal(l, i, M, R, beta, gam, SEED + 12, 0, sp)
        assert np.array_equal(g[i, :, :, :l.n], sp), f"instance {i}"
        assert np.array_equal(E[i], osE) and bE[i] == obE
        assert np.array_equal(bs[i, :l.n], obs)


@pytest.mark.parametrize("M", [8, 16, 64, 9])
def test_trotter_agreement_matches_oracle(M):
    """Correlation along the Trotter direction (agreement of every slice with slice 0) after an
    anneal, against the oracle: ragged site counts, three-colour lattices, R > 1."""
    insts = [_inst((5, 5, 5), 7, 41), _inst((7, 6, 3), 5, 42), _inst((9, 9, 9), 7, 43, 0, 0.2)]
    R = 3
    ctx = sg.sqa(insts, M, R, 3.0, SEED + 13)
    gam = linear_gamma(12)
    ctx.sqa_anneal(gam)
    got = ctx.trotter_agreement()
    for i, inst in enumerate(insts):
        l = _olat(inst)
        sp = oracle.sqa_init(l, i, M, R, SEED + 13)
        oracle.sqa_anneal(l, i, M, R, 3.0, gam, SEED + 13, 0, sp)
        assert np.array_equal(got[i], oracle.trotter_agreement(l, sp)), f"instance {i}"


def test_apt_with_fields_and_open_axes():
    insts = [_inst((5, 4, 3), 0, 11, hmax=3), _inst((6, 6, 6), 7, 12, hmax=31), _inst((3, 3, 3), 2, 13, hmax=1)]
    beta = geometric_ladder(6, 0.3, 2.0)
    ctx = sg.apt(insts, beta, SEED, reps_per_beta=2)
    with pytest.raises(sg.SGError) as e:
        ctx.icm(1.0)
    assert e.value.code == sg.SG_EUNSUPPORTED
    trace = ctx.run_apt(20, 2, float("inf"), record_every=4)
    g = ctx.spins()
    for i, inst in enumerate(insts):
        l = _olat(inst)
        sp = oracle.apt_init(l, i, 12, SEED)
        ctr = np.zeros(3, np.uint32)
        E = np.zeros(12, np.int64)
        b = np.array([np.iinfo(np.int64).max], np.int64)
        rc, otr, _ = oracle.apt_run(l, i, beta, 2, SEED, 20, 2, float("inf"), 4, ctr, sp, E, b)
        assert rc == 0
        assert np.array_equal(g[i, :, :l.n], sp) and np.array_equal(trace[i], otr)
    with pytest.raises(sg.SGError) as e:
        ctx.run_apt(2, 1, 1.5)
    assert e.value.code == sg.SG_EUNSUPPORTED


def test_apt_largest_lattices_multi_sweep_energy_sums():
    """Lattices near the 32767-site limit, one with fields up to 31 (75 threshold entries per
    slot) and one without (16 or fewer, tables in static LDS): one launch of three sweeps,
    whose per-sweep packed energy sums are at their largest (about 124 sites per thread)."""
    insts = [_inst((31, 32, 32), 7, 51, hmax=31), _inst((32, 32, 31), 7, 52)]
    beta = geometric_ladder(4, 0.3, 2.5)
    ctx = sg.apt(insts, beta, SEED, reps_per_beta=2)
    sb = np.repeat(beta, 2)
    ctx.sweep(3)
    g = ctx.spins()
    E = ctx.energy()
    for i, inst in enumerate(insts):
        l = _olat(inst)
        sp = oracle.apt_init(l, i, 8, SEED)
        for t in range(3):
            oracle.apt_sweep(l, i, sb, SEED, t, sp)
        assert np.array_equal(g[i, :, :l.n], sp), f"instance {i}"
        assert E[i].tolist() == [oracle.energy(l, s) for s in sp], f"instance {i}"


def test_apt_long_rows_use_queue_search():
    """x extent above 32 sites: the cluster search falls back to the breadth-first queue."""
    insts = [_inst((40, 3, 3), 7, 41), _inst((37, 2, 4), 5, 42), _inst((6, 6, 6), 7, 43)]
    beta = geometric_ladder(6, 0.4, 3.0)
    ctx = sg.apt(insts, beta, SEED, reps_per_beta=4)
    trace = ctx.run_apt(40, 1, 0.5, record_every=10)
    g = ctx.spins()
    for i, inst in enumerate(insts):
        l = _olat(inst)
        sp = oracle.apt_init(l, i, 24, SEED)
        ctr = np.zeros(3, np.uint32)
        E = np.zeros(24, np.int64)
        b = np.array([np.iinfo(np.int64).max], np.int64)
        rc, otr, _ = oracle.apt_run(l, i, beta, 4, SEED, 40, 1, 0.5, 10, ctr, sp, E, b)
        assert rc == 0 and np.array_equal(g[i, :, :l.n], sp) and np.array_equal(trace[i], otr)


def test_apt_queue_search_large_lattice():
    """Rows longer than 32 sites at a size where the LDS queue, the visited bits and the tile
    take about two thirds of the work-group's LDS (40 x 20 x 20 = 16000 sites), two labels."""
    insts = [_inst((40, 20, 20), 7, 71), _inst((33, 4, 5), 3, 72)]
    beta = geometric_ladder(4, 0.5, 3.0)
    ctx = sg.apt(insts, beta, SEED, reps_per_beta=2)
    trace = ctx.run_apt(6, 1, 0.5, record_every=2)
    g = ctx.spins()
    for i, inst in enumerate(insts):
        l = _olat(inst)
        sp = oracle.apt_init(l, i, 8, SEED)
        ctr = np.zeros(3, np.uint32)
        E = np.zeros(8, np.int64)
        b = np.array([np.iinfo(np.int64).max], np.int64)
        rc, otr, _ = oracle.apt_run(l, i, beta, 2, SEED, 6, 1, 0.5, 2, ctr, sp, E, b)
        assert rc == 0 and np.array_equal(g[i, :, :l.n], sp) and np.array_equal(trace[i], otr)
    assert ctx.energy()[0].tolist() == [oracle.energy(_olat(insts[0]), s) for s in g[0, :, :16000]]


def test_icm_rows_of_16_and_17_sites():
    """The cluster fill along x at the packing limit: rows of 16 sites fill both halves of a
    word with two pairs (the wrap bond at bit 15 and the boundary between the halves), open
    and periodic in x, and rows of 17 sites take one word per pair; four labels (two pairs per
    move) and two, cutoff low enough that most temperatures move."""
    insts = [_inst((16, 4, 4), 7, 91), _inst((16, 3, 5), 6, 92), _inst((17, 4, 3), 7, 93),
             _inst((16, 4, 3), 7, 94, p_absent=0.3)]
    beta = geometric_ladder(6, 0.3, 2.5)
    for reps in (4, 2):
        ctx = sg.apt(insts, beta, SEED + reps, reps_per_beta=reps)
        trace = ctx.run_apt(40, 1, 0.4, record_every=4)
        g = ctx.spins()
        for i, inst in enumerate(insts):
            l = _olat(inst)
            sp = oracle.apt_init(l, i, 6 * reps, SEED + reps)
            ctr = np.zeros(3, np.uint32)
            E = np.zeros(6 * reps, np.int64)
            b = np.array([np.iinfo(np.int64).max], np.int64)
            rc, otr, _ = oracle.apt_run(l, i, beta, reps, SEED + reps, 40, 1, 0.4, 4, ctr, sp, E, b)
            assert rc == 0 and np.array_equal(g[i, :, :l.n], sp), (reps, i)
            assert np.array_equal(trace[i], otr), (reps, i)
        ctx.close()


def test_apt_byte_offset_record_limit():
    """The sweep reads site records with neighbour byte offsets when every lattice of the
    context has at most 16383 sites (4 x 16383 fills 16 bits; on open axes an absent neighbour
    is the zero word after the last site, at offset 4 n), and site indices above that.  Each
    side of the limit in a context of its own: a 3 x 43 x 127 open lattice (16383 sites) and a
    32 x 32 x 16 periodic one (16384 sites), APT+ICM cycles against the oracle."""
    for shape, periodic, seed in (((3, 43, 127), 0, 81), ((32, 32, 16), 7, 82)):
        insts = [_inst(shape, periodic, seed)]
        beta = geometric_ladder(4, 0.5, 3.0)
        ctx = sg.apt(insts, beta, SEED, reps_per_beta=2)
        trace = ctx.run_apt(4, 1, 0.5, record_every=2)
        g = ctx.spins()
        l = _olat(insts[0])
        sp = oracle.apt_init(l, 0, 8, SEED)
        ctr = np.zeros(3, np.uint32)
        E = np.zeros(8, np.int64)
        b = np.array([np.iinfo(np.int64).max], np.int64)
        rc, otr, _ = oracle.apt_run(l, 0, beta, 2, SEED, 4, 1, 0.5, 2, ctr, sp, E, b)
        assert rc == 0 and np.array_equal(g[0, :, :l.n], sp), shape
        assert np.array_equal(trace[0], otr), shape
        assert ctx.energy()[0].tolist() == [oracle.energy(l, s) for s in sp], shape
        ctx.close()


@pytest.mark.parametrize("reps", [2, 4])
def test_apt_cluster_search_layouts(reps):
    """Row-bitset cluster search in both layouts: whole y-z planes per wave (wave-local fill:
    a wave filled exactly by 64-row planes, four waves of planes, open axes; rows of at most
    16 sites with both pairs packed in one word, 16 exactly, and 17 to 32 sites one word per
    pair) and one row per thread in thread order (more than 64 rows per plane, or more planes
    than four waves hold)."""
    insts = [_inst((2, 64, 4), 7, 61), _inst((5, 16, 16), 5, 62), _inst((5, 7, 9), 1, 63),
             _inst((4, 20, 20), 7, 64), _inst((3, 70, 2), 7, 65), _inst((7, 13, 20), 3, 66),
             _inst((16, 4, 4), 7, 67), _inst((20, 6, 6), 7, 68), _inst((32, 8, 8), 7, 69),
             _inst((17, 5, 12), 5, 70), _inst((20, 16, 16), 6, 71)]
    beta = geometric_ladder(6, 0.4, 3.0)
    ctx = sg.apt(insts, beta, SEED, reps_per_beta=reps)
    trace = ctx.run_apt(30, 1, 0.5, record_every=5)
    g = ctx.spins()
    for i, inst in enumerate(insts):
        l = _olat(inst)
        sp = oracle.apt_init(l, i, 6 * reps, SEED)
        ctr = np.zeros(3, np.uint32)
        E = np.zeros(6 * reps, np.int64)
        b = np.array([np.iinfo(np.int64).max], np.int64)
        rc, otr, _ = oracle.apt_run(l, i, beta, reps, SEED, 30, 1, 0.5, 5, ctr, sp, E, b)
        assert rc == 0 and np.array_equal(g[i, :, :l.n], sp), f"instance {i}"
        assert np.array_equal(trace[i], otr), f"instance {i}"


def test_paper_geometry_15x15x12_open_in_x_and_y():
    """The paper's logical-instance geometry (15 x 15 x 12, open in x and y, periodic in z):
    batched APT + ICM with 4 labels per temperature and DT-SQA at M = 64, sampled against
    the oracle."""
    insts = [(ej_couplings((15, 15, 12), 4, seed=70000 + i)[0], 4, None) for i in range(8)]
    beta = geometric_ladder(32, 0.2, 3.0)
    ctx = sg.apt(insts, beta, 99, 4)
    tr = ctx.run_apt(3, 1, 1.0, record_every=1)
    for i in (0, 7):
        l = oracle.Lattice(insts[i][0], 4)
        sp = oracle.apt_init(l, i, 128, 99)
        ctr = np.zeros(3, np.uint32)
        E = np.zeros(128, np.int64)
        b = np.array([np.iinfo(np.int64).max], np.int64)
        rc, otr, _ = oracle.apt_run(l, i, beta, 4, 99, 3, 1, 1.0, 1, ctr, sp, E, b)
        assert rc == 0 and np.array_equal(ctx.spins_range(i, 0, 128), sp), f"APT instance {i}"
        assert np.array_equal(tr[i], otr)
    q = sg.sqa(insts, 64, 16, 32.0, 98)
    q.sqa_anneal(linear_gamma(1000)[:3])
    for i, r in ((0, 0), (5, 15)):
        l = oracle.Lattice(insts[i][0], 4)
        sp = oracle.sqa_init(l, i, 64, 1, 98, r0=r)
        oracle.sqa_anneal(l, i, 64, 1, 32.0, linear_gamma(1000)[:3], 98, 0, sp, r0=r)
        assert np.array_equal(q.spins_range(i, r, 1)[0], sp[0]), f"DT-SQA instance {i} replica {r}"


def test_checkpoint_resume_is_exact():
    insts = [_inst(*m) for m in MIXED[:4]]
    beta = geometric_ladder(8, 0.2, 3.0)
    a = sg.apt(insts, beta, SEED, 2)
    a.run_apt(40, 1, 1.0)
    ref = a.spins()
    refE, refb = a.energy(), a.best()
    b = sg.apt(insts, beta, SEED, 2)
    b.run_apt(17, 1, 1.0)
    blob = b.get_state()
    c = sg.apt(insts, beta, SEED ^ 0xFFFF, 2)          # different seed: the blob restores the state, not the key
    c.set_state(blob)
    c2 = sg.apt(insts, beta, SEED, 2)
    c2.set_state(blob)
    c2.run_apt(23, 1, 1.0)
    assert np.array_equal(c2.spins(), ref)
    assert np.array_equal(c2.energy(), refE) and np.array_equal(c2.best(), refb)
    assert c2.counters().tolist() == [40, 40, 40]


@pytest.mark.parametrize("M", [8, 6, 2, 16, 32, 64, 3, 5, 7, 33, 63])
def test_sqa_matches_oracle(M):
    """DT-SQA against the oracle: initial state, spins after two anneal calls, slice energies
    and the minimum.  Odd M closes the Trotter ring between slices M - 1 and 0, both in word 0:
    three phases, the last slice updated on its own."""
    insts = [_inst((4, 4, 4), 7, 21), _inst((5, 5, 5), 7, 22), _inst((3, 4, 6), 3, 23),
             _inst((6, 6, 6), 7, 24, hmax=2), _inst((5, 3, 2), 0, 25, p_absent=0.2)]
    R, beta = 3, 2.0
    gam = linear_gamma(12, 3.0, 0.01)
    ctx = sg.sqa(insts, M, R, beta, SEED)
    lats = [_olat(x) for x in insts]
    g0 = ctx.spins()
    osp = [oracle.sqa_init(l, i, M, R, SEED) for i, l in enumerate(lats)]
    for i, l in enumerate(lats):
        assert np.array_equal(g0[i, :, :, :l.n], osp[i]), f"init {i}"
    bE, bs = ctx.sqa_anneal(gam[:7])
    bE2, bs2 = ctx.sqa_anneal(gam[7:])           # continues the step counter
    g = ctx.spins()
    sE = ctx.energy()
    for i, l in enumerate(lats):
        oracle.sqa_anneal(l, i, M, R, beta, gam[:7], SEED, 0, osp[i])
        obE, obs, osE = oracle.sqa_anneal(l, i, M, R, beta, gam[7:], SEED, 7, osp[i])
        assert np.array_equal(g[i, :, :, :l.n], osp[i]), f"instance {i}"
        assert np.array_equal(sE[i], osE)
        assert bE2[i] == obE and np.array_equal(bs2[i, :l.n], obs)
    assert ctx.counters()[0] == 12


def test_sqa_largest_lattice_in_lds():
    """A DT-SQA replica that nearly fills one work-group's LDS (19656 sites, 2 x 19665 words),
    with an open axis and fields, next to a small instance: spins, slice energies and the
    minimum after three steps; beyond the limit the context is refused."""
    insts = [_inst((28, 27, 26), 5, 61, hmax=3), _inst((4, 4, 4), 7, 62)]
    M, R, beta = 64, 2, 32.0
    gam = linear_gamma(3, 3.0, 0.01)
    ctx = sg.sqa(insts, M, R, beta, SEED)
    bE, _ = ctx.sqa_anneal(gam)
    g = ctx.spins()
    sE = ctx.energy()
    for i, inst in enumerate(insts):
        l = _olat(inst)
        sp = oracle.sqa_init(l, i, M, R, SEED)
        obE, _, osE = oracle.sqa_anneal(l, i, M, R, beta, gam, SEED, 0, sp)
        assert np.array_equal(g[i, :, :, :l.n], sp), f"instance {i}"
        assert np.array_equal(sE[i], osE) and bE[i] == obE
    with pytest.raises(sg.SGError) as e:
        sg.sqa([_inst((28, 28, 26), 5, 63)], M, R, beta, SEED)
    assert e.value.code == sg.SG_EUNSUPPORTED


def test_sqa_energy_without_schedule():
    """Slice energies right after creation and after a zero-step anneal: the kernel runs
    its energy pass with no threshold table."""
    insts = [_inst((5, 5, 5), 7, 51), _inst((4, 4, 4), 7, 52, hmax=3)]
    M, R = 8, 2
    ctx = sg.sqa(insts, M, R, 2.0, SEED)
    E0 = ctx.energy()
    bE, _ = ctx.sqa_anneal(np.zeros(0))
    g = ctx.spins()
    for i, inst in enumerate(insts):
        l = _olat(inst)
        sp = oracle.sqa_init(l, i, M, R, SEED)
        assert np.array_equal(g[i, :, :, :l.n], sp)
        ref = np.array([[oracle.energy(l, sp[r, k]) for k in range(M)] for r in range(R)])
        assert np.array_equal(E0[i], ref)
        assert bE[i] == ref.min()


SQA_THREADS = [192, 256, 320, 448, 512, 576, 768, 1024]


@pytest.mark.parametrize("hmax,M", [(0, 64), (6, 64), (20, 64), (0, 6), (20, 6), (0, 60), (0, 63),
                                    (20, 5)])
def test_sqa_every_launch_config_matches_oracle(hmax, M):
    """DT-SQA at several work-group sizes against the oracle, with threshold tables small
    enough to be pre-scaled (hmax 0), larger (6) and too large for double buffering (20);
    an odd number of steps; and the autotuner's pick."""
    insts = [_inst((5, 5, 5), 7, 41, hmax=hmax), _inst((4, 4, 6), 5, 42, hmax=hmax),
             _inst((3, 2, 5), 0, 43, hmax=hmax, p_absent=0.2 if hmax == 0 else 0.0)]
    R, beta = 2, 2.0
    gam = linear_gamma(9, 3.0, 0.01)
    lats = [_olat(x) for x in insts]
    ref = []
    for i, l in enumerate(lats):
        sp = oracle.sqa_init(l, i, M, R, SEED)
        obE, _, osE = oracle.sqa_anneal(l, i, M, R, beta, gam, SEED, 0, sp)
        ref.append((sp, osE, obE))
    for threads in SQA_THREADS + [0]:
        ctx = sg.sqa(insts, M, R, beta, SEED)
        ctx.set_launch_config(threads)
        assert ctx.launch_config() == threads
        bE, _ = ctx.sqa_anneal(gam)
        if threads == 0:
            assert ctx.launch_config() in (256, 512, 768, 1024)
        g = ctx.spins()
        sE = ctx.energy()
        for i, l in enumerate(lats):
            sp, osE, obE = ref[i]
            assert np.array_equal(g[i, :, :, :l.n], sp), f"threads {threads} instance {i}"
            assert np.array_equal(sE[i], osE) and bE[i] == obE, f"threads {threads} instance {i}"
        ctx.close()
    ctx = sg.sqa(insts, M, R, beta, SEED)
    for bad in (100, 64, 1088, -64):
        with pytest.raises(sg.SGError) as e:
            ctx.set_launch_config(bad)
        assert e.value.code == sg.SG_EINVAL


def test_adaptive_ladder_matches_oracle():
    """Few instances: the chains run as APT slots, four per work-group."""
    insts = [_inst((4, 4, 4), 7, 31), _inst((5, 5, 5), 7, 32), _inst((3, 4, 5), 7, 33)]
    kw = dict(beta0=0.5, alpha=1.25, tol=2.5, n_chains=10, sweeps=60, tail=25, max_steps=8)
    res = sg.adaptive_ladder(insts, SEED, **kw)
    for i, inst in enumerate(insts):
        ob, osg, _ = oracle.adaptive_ladder(_olat(inst), i, SEED, **kw)
        assert np.array_equal(res[i][0], ob), f"ladder {i}: {res[i][0]} vs {ob}"
        assert np.array_equal(res[i][1], osg)


@pytest.mark.parametrize("n_chains", [37, 64, 100, 32, 33])
def test_adaptive_ladder_chain_words(n_chains):
    """Chains 32 to a word (one work-group per instance and word, used once there are at least
    as many of them as CUs): a partial last word with a partial group (37), two full words (64),
    the Methods' 100 chains (three full words and one of four chains), one full word (32), and
    a full word with a last word of one chain (33)."""
    nw = (n_chains + 31) // 32
    n_inst = -(-256 // nw)
    shapes = [((4, 4, 4), 7), ((5, 4, 3), 0), ((2, 3, 7), 5), ((3, 3, 3), 7), ((6, 2, 2), 6)]
    insts = [_inst(shapes[i % 5][0], shapes[i % 5][1], 700 + i) for i in range(n_inst)]
    kw = dict(beta0=0.4, alpha=1.25, tol=2.0, n_chains=n_chains, sweeps=30, tail=15, max_steps=4)
    res = sg.adaptive_ladder(insts, SEED + 1, **kw)
    for i in sorted({0, 1, 2, 3, 4, n_inst - 1} | set(range(0, n_inst, 9))):
        ob, osg, _ = oracle.adaptive_ladder(_olat(insts[i]), i, SEED + 1, **kw)
        assert np.array_equal(res[i][0], ob), f"ladder {i}: {res[i][0]} vs {ob}"
        assert np.array_equal(res[i][1], osg)


def test_adaptive_ladder_with_fields():
    """Instances with fields run the chains as APT slots (byte per spin)."""
    insts = [_inst((4, 4, 4), 7, 44, hmax=2), _inst((3, 5, 4), 3, 45, hmax=1)]
    kw = dict(beta0=0.5, alpha=1.25, tol=2.5, n_chains=6, sweeps=40, tail=20, max_steps=5)
    res = sg.adaptive_ladder(insts, SEED + 2, **kw)
    for i, inst in enumerate(insts):
        ob, osg, _ = oracle.adaptive_ladder(_olat(inst), i, SEED + 2, **kw)
        assert np.array_equal(res[i][0], ob), f"ladder {i}: {res[i][0]} vs {ob}"
        assert np.array_equal(res[i][1], osg)


def test_mlp_gradient_matches_fp64_oracle():
    import ctypes as C
    lib = sg.load()
    rng = np.random.default_rng(4)
    P = np.zeros(sg.MLP_NPARAM + 8, np.float32)
    P[:sg.MLP_NPARAM] = rng.normal(0, 0.2, sg.MLP_NPARAM)
    mean = np.array([10.0, 2.0, 3.0, 0.5], np.float32)
    std = np.array([3.0, 0.5, 1.5, 0.05], np.float32)
    P[sg.MLP_NPARAM:sg.MLP_NPARAM + 4] = mean
    P[sg.MLP_NPARAM + 4:] = std
    x = (mean + std * rng.normal(0, 1, (37, 4))).astype(np.float32)
    y = rng.normal(0, 1, (37, 33)).astype(np.float32)
    h = C.c_void_p()
    assert lib.sg_mlp_create(P.ctypes.data_as(C.c_void_p), 1, None, C.byref(h)) == 0
    loss = C.c_float()
    grad = np.zeros(sg.MLP_NPARAM, np.float32)
    assert lib.sg_mlp_loss_grad(h, x.ctypes.data_as(C.c_void_p), y.ctypes.data_as(C.c_void_p), 37,
                                C.byref(loss), grad.ctypes.data_as(C.c_void_p)) == 0
    lib.sg_mlp_destroy(h)
    xs = (x.astype(np.float64) - mean) / std
    oloss, og, _ = oracle.mlp_loss_grad(P[:sg.MLP_NPARAM].astype(np.float64), xs, y.astype(np.float64))
    assert abs(loss.value - oloss) <= 1e-5 * abs(oloss) + 1e-7
    scale = np.abs(og).max()
    assert np.max(np.abs(grad - og)) <= 2e-5 * scale, np.max(np.abs(grad - og)) / scale


# --------------------------------------------------------------- full-size configurations
def test_plain_apt_L8_full_size_prefix():
    """L = 8 periodic, 32 betas geometric in [0.2, 3.0], 2 replicas per beta, ICM at beta >= 1."""
    J, _ = ej_couplings(8, 7, seed=1)
    beta = geometric_ladder(32, 0.2, 3.0)
    ctx = sg.apt([(J, 7, None)], beta, 1001, 2)
    tr = ctx.run_apt(40, 1, 1.0, record_every=1)
    l = oracle.Lattice(J, 7)
    sp = oracle.apt_init(l, 0, 64, 1001)
    ctr = np.zeros(3, np.uint32)
    E = np.zeros(64, np.int64)
    b = np.array([np.iinfo(np.int64).max], np.int64)
    _, otr, oacc = oracle.apt_run(l, 0, beta, 2, 1001, 40, 1, 1.0, 1, ctr, sp, E, b)
    assert np.array_equal(ctx.spins()[0], sp) and np.array_equal(tr[0], otr)
    assert np.array_equal(ctx.swap_counts()[0], oacc)


def test_batched_apt_256_mixed_sampled_instances():
    """256 instances, L round-robin over {6, 8, 10, 12, 15}, periodic, 32 betas x 2 replicas."""
    sizes = mixed_sizes(256)
    insts = [(ej_couplings(L, 7, seed=10000 + i)[0], 7, None) for i, L in enumerate(sizes)]
    beta = geometric_ladder(32, 0.2, 3.0)
    ctx = sg.apt(insts, beta, 777, 2)
    tr = ctx.run_apt(3, 1, 1.0, record_every=1)
    g = ctx.spins()
    for i in (0, 4, 9, 131, 254, 255):
        l = oracle.Lattice(insts[i][0], 7)
        sp = oracle.apt_init(l, i, 64, 777)
        ctr = np.zeros(3, np.uint32)
        E = np.zeros(64, np.int64)
        b = np.array([np.iinfo(np.int64).max], np.int64)
        _, otr, _ = oracle.apt_run(l, i, beta, 2, 777, 3, 1, 1.0, 1, ctr, sp, E, b)
        assert np.array_equal(g[i, :, :l.n], sp), f"instance {i} (L={sizes[i]})"
        assert np.array_equal(tr[i], otr)
    # properties that hold for every instance: energies are those of the returned states
    E = ctx.energy()
    for i in range(0, 256, 37):
        l = oracle.Lattice(insts[i][0], 7)
        assert E[i].tolist() == [oracle.energy(l, s[:l.n]) for s in g[i]]
    # the range reader returns the same logical slots
    for i, first, count in ((4, 0, 64), (131, 17, 5), (255, 63, 1)):
        assert np.array_equal(ctx.spins_range(i, first, count), g[i, first:first + count, :insts[i][0][..., 0].size])


@pytest.mark.parametrize("code", [13, 14, 15])
def test_batched_apt_256_mixed_two_launch_groups(code):
    """The 256-instance mixed batch with its replica kernels split into two launch groups on two
    streams (largest instances up to 65, 75 or 85 % of the sites, then the rest), over one
    32-cycle graph and a tail: sampled instances from both groups equal the oracle's."""
    sizes = mixed_sizes(256)
    insts = [(ej_couplings(L, 7, seed=10000 + i)[0], 7, None) for i, L in enumerate(sizes)]
    beta = geometric_ladder(32, 0.2, 3.0)
    ctx = sg.apt(insts, beta, 779, 2)
    ctx.set_launch_config(code)
    tr = ctx.run_apt(35, 1, 1.0, record_every=5)
    g = ctx.spins()
    cnt = ctx.swap_counts()
    for i in (0, 1, 2, 3, 4, 128, 255):
        l = oracle.Lattice(insts[i][0], 7)
        sp = oracle.apt_init(l, i, 64, 779)
        ctr = np.zeros(3, np.uint32)
        E = np.zeros(64, np.int64)
        b = np.array([np.iinfo(np.int64).max], np.int64)
        _, otr, oacc = oracle.apt_run(l, i, beta, 2, 779, 35, 1, 1.0, 5, ctr, sp, E, b)
        assert np.array_equal(g[i, :, :l.n], sp), f"config {code}, instance {i} (L={sizes[i]})"
        assert np.array_equal(tr[i], otr) and np.array_equal(cnt[i], oacc), f"config {code}, instance {i}"


def test_sqa_L10_M32_R64_sampled_replicas():
    """L = 10 periodic, M = 32, R = 64, beta = 4, Gamma 3.0 -> 0.01 over 2000 steps (prefix)."""
    J, _ = ej_couplings(10, 7, seed=1)
    gam = linear_gamma(2000)
    ctx = sg.sqa([(J, 7, None)], 32, 64, 4.0, 2002)
    ctx.sqa_anneal(gam[:6])
    g = ctx.spins()
    l = oracle.Lattice(J, 7)
    for r in (0, 17, 63):
        sp = oracle.sqa_init(l, 0, 32, 1, 2002, r0=r)
        oracle.sqa_anneal(l, 0, 32, 1, 4.0, gam[:6], 2002, 0, sp, r0=r)
        assert np.array_equal(g[0, r, :, :], sp[0]), f"replica {r}"


def test_sqa_L15_M64_R1024_sampled_replicas_benchmark_configuration():
    """The timed workload itself: 32 instances of L = 15, M = 64, R = 1024, beta = 32, in the
    launch configuration the autotuner picks; sampled replicas against the oracle."""
    insts = [(ej_couplings(15, 7, seed=20000 + i)[0], 7, None) for i in range(32)]
    gam = linear_gamma(1000)
    ctx = sg.sqa(insts, 64, 1024, 32.0, 4004)
    bE, _ = ctx.sqa_anneal(gam[:4])
    assert ctx.launch_config() in (256, 512, 768, 1024)
    sE = ctx.energy()
    for i, r in ((0, 0), (17, 511), (31, 1023)):
        l = oracle.Lattice(insts[i][0], 7)
        sp = oracle.sqa_init(l, i, 64, 1, 4004, r0=r)
        _, _, osE = oracle.sqa_anneal(l, i, 64, 1, 32.0, gam[:4], 4004, 0, sp, r0=r)
        assert np.array_equal(ctx.spins_range(i, r, 1)[0], sp[0]), f"instance {i} replica {r}"
        assert np.array_equal(sE[i, r], osE[0])
    assert np.array_equal(bE, sE.reshape(32, -1).min(axis=1))
    with pytest.raises(sg.SGError) as e:
        ctx.spins_range(0, 1020, 5)
    assert e.value.code == sg.SG_EINVAL


def test_sqa_L15_M64_R64_sampled_replicas():
    """32 instances of L = 15 periodic (three colours), M = 64, R = 64, beta = 32."""
    insts = [(ej_couplings(15, 7, seed=20000 + i)[0], 7, None) for i in range(32)]
    gam = linear_gamma(1000)
    ctx = sg.sqa(insts, 64, 64, 32.0, 4004)
    bE, _ = ctx.sqa_anneal(gam[:3])
    g = ctx.spins()
    sE = ctx.energy()
    for i, r in ((0, 0), (13, 40), (31, 63)):
        l = oracle.Lattice(insts[i][0], 7)
        sp = oracle.sqa_init(l, i, 64, 1, 4004, r0=r)
        _, _, osE = oracle.sqa_anneal(l, i, 64, 1, 32.0, gam[:3], 4004, 0, sp, r0=r)
        assert np.array_equal(g[i, r], sp[0]), f"instance {i} replica {r}"
        assert np.array_equal(sE[i, r], osE[0])
    assert np.array_equal(bE, sE.reshape(32, -1).min(axis=1))


def test_degenerate_lattices():
    """A single site, axes of length one and two, and a lattice with every bond absent:
    APT + ICM and DT-SQA against the oracle (and one small instance with fields, without ICM)."""
    plain = [_inst((1, 1, 1), 7, 81), _inst((2, 1, 1), 1, 82), _inst((1, 5, 1), 2, 83),
             _inst((3, 3, 3), 7, 84, p_absent=1.0)]
    fields = [_inst((2, 2, 2), 7, 85, hmax=2)]
    beta = geometric_ladder(4, 0.3, 2.0)
    for insts, cut in ((plain, 0.5), (fields, float("inf"))):
        ctx = sg.apt(insts, beta, SEED, reps_per_beta=2)
        trace = ctx.run_apt(40, 1, cut, record_every=4)
        g = ctx.spins()
        for i, inst in enumerate(insts):
            l = _olat(inst)
            sp = oracle.apt_init(l, i, 8, SEED)
            ctr = np.zeros(3, np.uint32)
            E = np.zeros(8, np.int64)
            b = np.array([np.iinfo(np.int64).max], np.int64)
            rc, otr, _ = oracle.apt_run(l, i, beta, 2, SEED, 40, 1, cut, 4, ctr, sp, E, b)
            assert rc == 0 and np.array_equal(g[i, :, :l.n], sp), f"instance {i}"
            assert np.array_equal(trace[i], otr), f"instance {i}"
    insts = plain + fields
    q = sg.sqa(insts, 8, 2, 2.0, SEED)
    gam = linear_gamma(6)
    bE, _ = q.sqa_anneal(gam)
    for i, inst in enumerate(insts):
        l = _olat(inst)
        s5 = oracle.sqa_init(l, i, 8, 2, SEED)
        obE, _, _ = oracle.sqa_anneal(l, i, 8, 2, 2.0, gam, SEED, 0, s5)
        assert np.array_equal(q.spins()[i, :, :, :l.n], s5) and bE[i] == obE, f"instance {i}"


class _DevBuf:
    """Device memory from the HIP runtime that libsg itself uses (found among the process's
    loaded libraries), for the device-output calls; filled with 7 so that unwritten entries
    show."""

    _hip = None

    def __init__(self, shape, dtype):
        import ctypes
        if _DevBuf._hip is None:
            sg.load()
            path = next(line.split()[-1] for line in open("/proc/self/maps")
                        if "libamdhip64" in line)
            _DevBuf._hip = ctypes.CDLL(path)
        self.shape, self.dtype = tuple(shape), np.dtype(dtype)
        self.nbytes = int(np.prod(self.shape)) * self.dtype.itemsize
        self.ptr = ctypes.c_void_p()
        assert _DevBuf._hip.hipMalloc(ctypes.byref(self.ptr), ctypes.c_size_t(self.nbytes)) == 0
        fill = np.full(self.shape, 7, self.dtype)
        assert _DevBuf._hip.hipMemcpy(self.ptr, fill.ctypes.data_as(ctypes.c_void_p),
                                      ctypes.c_size_t(self.nbytes), 1) == 0   # host to device

    def data_ptr(self):
        return self.ptr.value

    def numpy(self):
        import ctypes
        out = np.empty(self.shape, self.dtype)
        assert _DevBuf._hip.hipMemcpy(out.ctypes.data_as(ctypes.c_void_p), self.ptr,
                                      ctypes.c_size_t(self.nbytes), 2) == 0   # device to host
        return out

    def free(self):
        if self.ptr:
            _DevBuf._hip.hipFree(self.ptr)
            self.ptr = None


def test_device_outputs_equal_the_host_calls():
    """The device-output calls write the host calls' results, bit for bit, into device memory:
    APT energies, spins (through the slot mapping after exchanges) and running minima after
    cycles; DT-SQA (even and odd M) the anneal's minimum and state from a twin context with the
    same seed, then slice energies and spins.  Host addresses are refused before any work."""
    insts = [_inst((5, 5, 5), 7, 71), _inst((4, 6, 3), 5, 72), _inst((6, 6, 6), 7, 73, p_absent=0.1)]
    ctx = sg.apt(insts, geometric_ladder(8, 0.3, 2.0), SEED, reps_per_beta=2)
    ctx.run_apt(20, 1, 1.0)
    E, S, B = ctx.energy(), ctx.spins(), ctx.best()
    bufs = [_DevBuf(E.shape, np.int64), _DevBuf(S.shape, np.int8), _DevBuf(B.shape, np.int64)]
    ctx.energy_dev(bufs[0])
    ctx.spins_dev(bufs[1])
    ctx.best_dev(bufs[2])
    ctx.synchronize()
    assert np.array_equal(bufs[0].numpy(), E)
    assert np.array_equal(bufs[1].numpy(), S)
    assert np.array_equal(bufs[2].numpy(), B)
    host = np.zeros(S.size, np.int64)
    for call in (ctx.energy_dev, ctx.best_dev, ctx.spins_dev):
        with pytest.raises(sg.SGError) as e:
            call(host.ctypes.data)
        assert e.value.code == sg.SG_EINVAL
    assert np.array_equal(ctx.energy(), E)                      # the refusals changed nothing
    ctx.close()
    for b in bufs:
        b.free()
    for M in (8, 7):
        gam = linear_gamma(9)
        ca = sg.sqa(insts, M, 3, 2.0, SEED + 21)
        cb = sg.sqa(insts, M, 3, 2.0, SEED + 21)
        bE, bs = ca.sqa_anneal(gam)
        sE, sS = ca.energy(), ca.spins()
        bufs = [_DevBuf(bE.shape, np.int64), _DevBuf(bs.shape, np.int8), _DevBuf(sE.shape, np.int64),
                _DevBuf(sS.shape, np.int8)]
        cb.sqa_anneal_dev(gam, bufs[0], bufs[1])
        cb.energy_dev(bufs[2])
        cb.spins_dev(bufs[3])
        cb.synchronize()
        for got, want in zip(bufs, (bE, bs, sE, sS)):
            assert np.array_equal(got.numpy(), want), M
            got.free()
        ca.close()
        cb.close()


def test_device_allocation_failure_is_reported():
    """A DT-SQA context whose replicas need more than the device's memory (256 L = 15 instances
    x 65535 replicas x 27 KB = 453 GB, inside the replica-count limit) fails at its allocation
    with SG_ENOMEM and a message, before any kernel runs; the device then serves a small
    context exactly as before."""
    from paper_2503_10302_amd.inputs import ej_couplings
    J, _ = ej_couplings(15, 7, seed=5)
    with pytest.raises(sg.SGError) as e:
        sg.sqa([(J, 7, None)] * 256, 64, 65535, 32.0, SEED)
    assert e.value.code == sg.SG_ENOMEM
    assert "out of device memory" in str(e.value)
    inst = _inst((4, 4, 4), 7, 81)
    ctx = sg.sqa([inst], 8, 2, 2.0, SEED)
    gam = linear_gamma(5)
    bE, _ = ctx.sqa_anneal(gam)
    l = _olat(inst)
    sp = oracle.sqa_init(l, 0, 8, 2, SEED)
    obE, _, _ = oracle.sqa_anneal(l, 0, 8, 2, 2.0, gam, SEED, 0, sp)
    assert np.array_equal(ctx.spins()[0, :, :, :l.n], sp) and bE[0] == obE
    ctx.close()


def test_invalid_calls_leave_the_context_unchanged():
    """SG_EINVAL leaves a context as it was: invalid calls on an APT and a DT-SQA context are
    each refused and change neither spins, energies, counters, running minima nor swap counts,
    and both contexts then continue exactly like twins that never saw the calls."""
    insts = [_inst((5, 5, 5), 7, 91), _inst((4, 4, 6), 5, 92)]
    beta = geometric_ladder(8, 0.3, 2.0)
    a, ta = sg.apt(insts, beta, SEED, 2), sg.apt(insts, beta, SEED, 2)
    a.run_apt(10, 1, 1.0)
    ta.run_apt(10, 1, 1.0)

    def snap(c):
        return (c.spins(), c.energy(), c.counters(), c.best(), c.swap_counts())

    before = snap(a)
    bad = [lambda: a.sweep(-1), lambda: a.run_apt(5, 0, 1.0), lambda: a.run_apt(-1, 1, 1.0),
           lambda: a.run_apt_ex(5, 1, 1.0, icm_pairs=3), lambda: a.run_apt_ex(5, 1, float("nan")),
           lambda: a.icm_ex(1.0, icm_pairs=0), lambda: a.set_spins(np.zeros_like(before[0])),
           lambda: a.set_state(np.zeros(7, np.uint8)), lambda: a.set_launch_config(99)]
    for k, f in enumerate(bad):
        with pytest.raises(sg.SGError) as e:
            f()
        assert e.value.code == sg.SG_EINVAL, k
    for x, y in zip(before, snap(a)):
        assert np.array_equal(x, y)
    a.run_apt(10, 1, 1.0)
    ta.run_apt(10, 1, 1.0)
    for x, y in zip(snap(a), snap(ta)):
        assert np.array_equal(x, y)
    a.close()
    ta.close()

    s, ts = sg.sqa(insts, 8, 2, 2.0, SEED), sg.sqa(insts, 8, 2, 2.0, SEED)
    g = linear_gamma(6)
    s.sqa_anneal(g[:3])
    ts.sqa_anneal(g[:3])

    def snap2(c):
        return (c.spins(), c.energy(), c.counters())

    before = snap2(s)
    zero = g[3:].copy()
    zero[1] = 0.0
    bad = [lambda: s.sqa_anneal(zero), lambda: s.sqa_anneal(np.array([np.nan])),
           lambda: s.set_spins(np.zeros_like(before[0])), lambda: s.set_launch_config(100),
           lambda: s.set_state(np.zeros(3, np.uint8))]
    for k, f in enumerate(bad):
        with pytest.raises(sg.SGError) as e:
            f()
        assert e.value.code == sg.SG_EINVAL, k
    for x, y in zip(before, snap2(s)):
        assert np.array_equal(x, y)
    bE, bs = s.sqa_anneal(g[3:])
    tE, tsb = ts.sqa_anneal(g[3:])
    assert np.array_equal(bE, tE) and np.array_equal(bs, tsb)
    for x, y in zip(snap2(s), snap2(ts)):
        assert np.array_equal(x, y)
    s.close()
    ts.close()
