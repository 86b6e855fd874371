"""Host-side checks of libsg that need no GPU: exports, argument validation, loud failure."""
import os
import re

import numpy as np
import pytest

from paper_2503_10302_amd import sg
from paper_2503_10302_amd.inputs import ej_couplings, geometric_ladder

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "sg.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sg_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import subprocess
    lib = sg.load()
    names = _declared()
    assert len(names) >= 25
    for nm in names:
        assert hasattr(lib, nm), nm
    out = subprocess.run(["nm", "-D", "--defined-only", sg.SO_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    assert set(names) <= exported
    assert set(sg.EXPORTS) == set(names)


def _expect(code, fn):
    with pytest.raises(sg.SGError) as e:
        fn()
    assert e.value.code == code, str(e.value)


def test_invalid_arguments_are_rejected_before_any_device_work():
    J, _ = ej_couplings(4, 7, seed=1)
    beta = geometric_ladder(8)
    _expect(sg.SG_EINVAL, lambda: sg.apt([(J, 7, None)], beta[::-1].copy(), 1, 2))      # descending
    _expect(sg.SG_EINVAL, lambda: sg.apt([(J, 7, None)], beta, 1, 3))                    # labels
    _expect(sg.SG_EINVAL, lambda: sg.apt([(J, 7, None)], beta[:1], 1, 2))                # one beta
    Jbad = J.copy(); Jbad[0, 0, 0, 0] = 2
    _expect(sg.SG_EINVAL, lambda: sg.apt([(Jbad, 7, None)], beta, 1, 2))                 # |J| > 1
    h = np.full(64, 40, np.int8)
    _expect(sg.SG_EINVAL, lambda: sg.apt([(J, 7, h)], beta, 1, 2))                       # |h| > 31
    Jbig = np.ones((40, 40, 40, 3), np.int8)
    _expect(sg.SG_EINVAL, lambda: sg.apt([(Jbig, 7, None)], beta, 1, 2))                 # n too large
    _expect(sg.SG_EINVAL, lambda: sg.sqa([(J, 7, None)], 65, 2, 1.0, 1))                 # M > 64
    _expect(sg.SG_EINVAL, lambda: sg.sqa([(J, 7, None)], 1, 2, 1.0, 1))                  # M < 2
    _expect(sg.SG_EINVAL, lambda: sg.sqa([(J, 7, None)], 8, 0, 1.0, 1))                  # R = 0
    _expect(sg.SG_EINVAL, lambda: sg.sqa([(J, 7, None)], 8, 2, -1.0, 1))                 # beta <= 0


def test_lowest_invalid_instance_is_reported():
    """Instances are checked and their tables built on several host threads; with several
    invalid instances the error names the lowest of them, whatever the threads' timing."""
    beta = geometric_ladder(8)
    insts = []
    for i in range(64):
        J, _ = ej_couplings(5, 7, seed=100 + i)
        if i in (9, 23, 41, 60):
            J = J.copy()
            J[1, 2, 3, i % 3] = 2
        insts.append((J, 7, None))
    for _ in range(20):
        with pytest.raises(sg.SGError) as e:
            sg.apt(insts, beta, 1, 2)
        assert e.value.code == sg.SG_EINVAL and "instance 9:" in str(e.value), str(e.value)
        with pytest.raises(sg.SGError) as e:
            sg.sqa(insts, 8, 2, 4.0, 1)
        assert e.value.code == sg.SG_EINVAL and "instance 9:" in str(e.value), str(e.value)


def test_no_silent_cpu_fallback():
    """Valid input on a machine without a GPU fails with SG_EHIP instead of computing elsewhere."""
    J, _ = ej_couplings(4, 7, seed=1)
    try:
        ctx = sg.apt([(J, 7, None)], geometric_ladder(8), 1, 2)
    except sg.SGError as e:
        assert e.code == sg.SG_EHIP
        return
    ctx.close()
    pytest.skip("a GPU is present; this check is for hosts without one")


def test_binding_module_has_no_oracle_import():
    import paper_2503_10302_amd
    pkg = os.path.dirname(paper_2503_10302_amd.__file__)
    for root, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(root, f)).read()
                assert "import oracle" not in txt and "sg_oracle" not in txt and "sgo_" not in txt, f


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs the whole path on one GPU and says so when asked for more."""
    import subprocess
    import sys
    root = os.path.dirname(HEADER).rsplit(os.sep, 1)[0]
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bench_roofline_accounting():
    """The roofline inputs of the benchmark: 17.4 algorithmic slots per DT-SQA flip at 64
    slices (65 per four-slice group, 5 per site and parity shared by the eight groups, one
    compare per slice), the MI355X VALU peak, and HBM counters reported only for the kernel
    source, replica count and step count they were measured on."""
    import importlib.util
    root = os.path.dirname(HEADER).rsplit(os.sep, 1)[0]
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    assert abs(b.alg_ops_per_flip(8) - (65 / 4 + 5 / 32 + 1)) < 1e-12
    assert abs(b.VALU_PEAK_TOPS - 78.6432) < 1e-9
    t = b.SQA_TRAFFIC
    current = b.sqa_kernel_source_hash() == t["kernel_src_sha256_16"]
    for steps, m in t["by_steps"].items():
        v = b.sqa_traffic(t["R"], steps)
        if current:
            assert v == round((m["fetch_kib"] * t["fetch_scale"] + m["write_kib"] * t["write_scale"]) * 1024)
        else:
            assert v is None   # counters taken on another version of the kernel are not reported
        assert b.sqa_traffic(t["R"] // 2, steps) is None
    assert b.sqa_traffic(t["R"], 1 + max([0] + list(t["by_steps"]))) is None


def test_instance_features_equal_the_oracle():
    """sg_instance_features (host code of the library, input of the ladder network) against
    the oracle's sgo_instance_features, exactly: periodic, open, mixed-boundary, diluted and
    thin lattices, with and without fields (fields are not features)."""
    import oracle
    from paper_2503_10302_amd import ladder
    from paper_2503_10302_amd.inputs import diluted_couplings
    cases = []
    for k, (shape, per) in enumerate([((8, 8, 8), 7), ((15, 15, 15), 7), ((15, 15, 12), 4),
                                      ((6, 7, 5), 0), ((9, 4, 3), 5), ((2, 2, 2), 7),
                                      ((1, 1, 6), 4), ((10, 10, 10), 3)]):
        J, h = ej_couplings(shape, per, seed=300 + k, h_max=3 if k % 3 == 0 else 0)
        cases.append((J, per, h))
        cases.append((diluted_couplings(shape, per, seed=400 + k, p_absent=0.2), per, None))
    got = ladder.features(cases)
    for i, (J, per, h) in enumerate(cases):
        want = oracle.instance_features(oracle.Lattice(J, per, h))
        assert got[i].tolist() == want.tolist(), (i, got[i], want)


def test_flips_per_ns_is_the_papers_count():
    """The benchmark's throughput is the paper's: one flip is one update attempt of one spin,
    so a sweep of n p-bits in t ns gives n / t flips/ns.  The paper's FPGA figures: 2687 and
    4096 p-bits per 22.22 ns sweep are 120.9 and 184.3 flips/ns."""
    import bench
    assert abs(bench.flips_per_ns(2687, 22.22e-6) - 120.9) < 0.05
    assert abs(bench.flips_per_ns(4096, 22.22e-6) - 184.3) < 0.05
    # one DT-SQA step of the headline workload: 32 instances x R replicas x M slices x 15^3
    assert bench.flips_per_ns(32 * 1024 * 64 * 3375, 2.64) == 32 * 1024 * 64 * 3375 / 2.64e6


def test_threshold_builders_equal_the_oracle():
    """The library's FP64 threshold builders (the code that fills every context's tables) give
    the oracle's thresholds exactly, over the inverse temperatures and fields of the workloads
    and beyond: the heat bath for the geometric ladders, adaptive-like ladders and fields up to
    31; DT-SQA for M = 2..64 (odd included), beta = M / 2 and 4, every Gamma of 2000-step
    linear schedules, fields up to 6 + 31 and every Trotter sum; the swap rule for random
    ladder pairs, unfavourable energy changes and uniform words (the oracle decides the
    exchange, the library's threshold must decide it the same way)."""
    import oracle
    from paper_2503_10302_amd import sg
    from paper_2503_10302_amd.inputs import geometric_ladder, linear_gamma
    oracle.build()
    rng = np.random.default_rng(17)
    betas = np.concatenate([geometric_ladder(32, 0.2, 3.0), geometric_ladder(8, 0.3, 2.0),
                            np.cumsum(rng.uniform(0.01, 0.3, 40)) + 0.5, [0.0, 1e-9, 30.0]])
    for b in betas:
        for I in range(-37, 38):
            assert sg.threshold_heat_bath(b, I) == oracle.heat_threshold(b, I), (b, I)
    for M in (2, 3, 7, 16, 32, 33, 63, 64):
        for beta in (M / 2.0, 4.0):
            gam = linear_gamma(2000)[rng.choice(2000, 60, replace=False)]
            for g in np.concatenate([gam, [3.0, 0.01]]):
                for s_ in (-37, -6, -2, 0, 1, 2, 6, 37):
                    for tau in (-2, 0, 2):
                        assert (sg.threshold_sqa(beta, M, g, s_, tau) ==
                                oracle.sqa_threshold(beta, M, g, s_, tau)), (M, beta, g, s_, tau)
    lad = geometric_ladder(32, 0.2, 3.0)
    for _ in range(3000):
        k = int(rng.integers(0, 31))
        d = int(rng.integers(1, 400))
        u = int(rng.integers(0, 2 ** 32))
        T = sg.threshold_swap(lad[k], lad[k + 1], d)
        assert (u < T) == bool(oracle.swap_accept(lad[k], lad[k + 1], 0, -d, u)), (k, d, u)
