"""Planted mistakes: each test builds a copy of the oracle with one plausible mistake (a
wrong sign, a dropped term, a wrong factor or index) and checks that the oracle's pin suite
(tests/test_oracle_basic.py, tests/test_oracle_sampling.py, tests/test_colouring_cpu.py) fails
against it.  The mutated
copies live in a temporary directory; the oracle itself is untouched."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sg_oracle.c")
HDR = os.path.join(ROOT, "oracle", "sg_oracle.h")

MUTANTS = [
    ("philox_nine_rounds", "for (int round = 0; round < 10; ++round) {",
     "for (int round = 0; round < 9; ++round) {"),
    ("philox_key_schedule", "            k1 += W1;", "            k1 += W0;"),
    ("heat_bath_factor_two", "    double x = beta * (double)I;\n    double p = 0.5 * (1.0 + tanh(x));",
     "    double x = beta * (double)I;\n    double p = 0.5 * (1.0 + tanh(2.0 * x));"),
    ("swap_sign", "double x = (beta_hi - beta_lo) * (double)(E_hi - E_lo);",
     "double x = (beta_hi - beta_lo) * (double)(E_lo - E_hi);"),
    ("swap_alternation", "int32_t first = (a & 1u) ? 0 : 1;", "int32_t first = (a & 1u) ? 1 : 0;"),
    ("field_drops_z_bonds", "            if (nb >= 0) I += sgo_bond(lat, j, a, dir) * s[nb];",
     "            if (nb >= 0 && a < 2) I += sgo_bond(lat, j, a, dir) * s[nb];"),
    ("energy_drops_z_bonds", "            if (nb >= 0) E -= (int64_t)lat->J[3 * j + a] * s[j] * s[nb];",
     "            if (nb >= 0 && a < 2) E -= (int64_t)lat->J[3 * j + a] * s[j] * s[nb];"),
    ("colouring_odd_ring_label",
     "if (C == 3 && odd_ring(lat, a) && c == axis_len(lat, a) - 1) sum += 2;",
     "if (C == 3 && odd_ring(lat, a) && c == axis_len(lat, a) - 1) sum += 0;"),
    ("jperp_methods_factor", "double K = -0.5 * log(tanh(beta * gamma / (double)M));",
     "double K = -1.0 * log(tanh(beta * gamma / (double)M));"),
    ("trotter_one_neighbour", "uint32_t T = sgo_sqa_threshold(beta, M, gamma, s, up + dn);",
     "uint32_t T = sgo_sqa_threshold(beta, M, gamma, s, 2 * up);"),
    ("icm_ignores_overlap", "if (inC[nb] || A[nb] == B[nb]) continue;", "if (inC[nb]) continue;"),
    ("icm_never_big_cluster", "            if (2 * size > n) {", "            if (size > n) {"),
    ("icm_cluster_in_one_replica", "                    B[j] = (int8_t)-B[j];\n", ""),
    ("adaptive_sigma_biased", "double sigma = sum / (double)nc;",
     "double sigma = 1.05 * sum / (double)nc;"),
    ("adaptive_variance_for_std", "    return sqrt(var);", "    return var;"),
    ("mlp_drops_softplus_slope", "dO[i] = sigmoid(o[i]) * suffix;", "dO[i] = suffix;"),
    ("apt_init_biased_threshold", "spins[(int64_t)s * n + j] = (w < 0x80000000u) ? 1 : -1;",
     "spins[(int64_t)s * n + j] = (w < 0x40000000u) ? 1 : -1;"),
    ("apt_init_one_word_per_block",
     "uint32_t w = sgo_word(seed, (uint32_t)j, 0u, (uint32_t)s >> 2, inst, tag, s & 3);",
     "uint32_t w = sgo_word(seed, (uint32_t)j, 0u, (uint32_t)s >> 2, inst, tag, 0);"),
    ("sqa_init_biased_threshold", "spins[((int64_t)r * M + k) * n + j] = (w < 0x80000000u) ? 1 : -1;",
     "spins[((int64_t)r * M + k) * n + j] = (w < 0x40000000u) ? 1 : -1;"),
    ("sqa_init_one_word_per_block", "SGO_TAG_SQA_INIT, (k >> 1) & 3);", "SGO_TAG_SQA_INIT, 0);"),
    ("colour_map_drops_trotter_label", "if (lat->colour) return (lat->colour[j] + trotter_label(M, k)) % C;",
     "if (lat->colour) return lat->colour[j] % C;"),
    ("trotter_agreement_with_previous_slice", "const int8_t *s0 = spins + ((int64_t)r * M) * n;",
     "const int8_t *s0 = spins + ((int64_t)r * M + (k > 0 ? k - 1 : 0)) * n;"),
    ("icm_one_pair_always_first",
     "only = (int32_t)(sgo_word(seed, (uint32_t)b, a, 0u, inst, SGO_TAG_ICM_PAIR, 1) >> 31);",
     "only = 0;"),
]


def _run_mutant(tmp, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"{name}: the planted site is not unique"
    d = os.path.join(tmp, name)
    os.makedirs(d)
    with open(os.path.join(d, "sg_oracle.c"), "w") as f:
        f.write(src.replace(old, new))
    with open(os.path.join(d, "sg_oracle.h"), "w") as f:
        f.write(open(HDR).read())
    so = os.path.join(d, "liboracle_mutant.so")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                           "-shared", "-o", so, os.path.join(d, "sg_oracle.c"), "-lm"])
    env = dict(os.environ, SG_ORACLE_SO=so, PYTHONDONTWRITEBYTECODE="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "tests/test_oracle_basic.py", "tests/test_oracle_sampling.py",
                        "tests/test_colouring_cpu.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    failed = [l for l in r.stdout.splitlines() if l.startswith("FAILED")]
    return name, r.returncode, failed[:1]


def test_every_planted_mistake_fails_the_pins(tmp_path):
    with ThreadPoolExecutor(max_workers=6) as ex:
        results = list(ex.map(lambda m: _run_mutant(str(tmp_path), *m), MUTANTS))
    missed = [name for name, rc, _ in results if rc == 0]
    for name, rc, failed in results:
        print(f"{name}: exit {rc} {failed}")
    assert not missed, f"pins did not catch: {missed}"
    # an exit status of 1 means tests failed (not an error in collection or a crash)
    assert all(rc == 1 for _, rc, _ in results), results


def test_unmutated_copy_passes_the_pins(tmp_path):
    """Control: the same procedure on an unmodified copy passes (the mutants fail because
    of the planted mistake, not because of the procedure)."""
    name, rc, failed = _run_mutant(str(tmp_path), "control", "/* Thresholds.", "/* Thresholds.")
    assert rc == 0, failed
