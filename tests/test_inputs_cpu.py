"""The seeded input generators: the structure of the paper's workloads (Eq. 1: +-1
nearest-neighbour couplings with equal probability; the linear field ramp of the DT-SQA
schedule; geometric temperature ladders), reproducible from their seeds."""
import numpy as np

from paper_2503_10302_amd.inputs import (diluted_couplings, ej_couplings, geometric_ladder,
                                         linear_gamma, mixed_sizes)


def test_couplings_are_plus_minus_one_with_equal_probability():
    J, h = ej_couplings(15, 7, seed=3)
    assert h is None and J.shape == (15, 15, 15, 3) and J.dtype == np.int8
    assert set(np.unique(J)) == {-1, 1}
    n = J.size
    # a binomial count within 5 standard deviations of n / 2
    assert abs(int((J > 0).sum()) - n / 2) < 5 * np.sqrt(n / 4)


def test_open_axes_have_no_boundary_bonds():
    J, _ = ej_couplings((5, 4, 3), periodic=0b010, seed=1)   # only y periodic
    assert np.all(J[:, :, 4, 0] == 0) and np.all(J[2, :, :, 2] == 0)   # +x at x = 4, +z at z = 2
    assert np.all(J[:, :, :4, 0] != 0) and np.all(J[:, 3, :, 1] != 0)  # interior x, periodic y
    J1, _ = ej_couplings((1, 3, 3), periodic=7, seed=1)             # an axis of length one
    assert np.all(J1[..., 0] == 0)


def test_seeds_reproduce_and_differ():
    a, _ = ej_couplings(6, 7, seed=10)
    b, _ = ej_couplings(6, 7, seed=10)
    c, _ = ej_couplings(6, 7, seed=11)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_fields_and_dilution():
    _, h = ej_couplings(8, 7, seed=2, h_max=3)
    assert h.shape == (512,) and h.min() >= -3 and h.max() <= 3 and len(np.unique(h)) == 7
    J = diluted_couplings(12, 7, seed=4, p_absent=0.25)
    frac = float((J == 0).mean())
    assert abs(frac - 0.25) < 0.02


def test_ladders_ramps_and_batch_sizes():
    b = geometric_ladder(32, 0.2, 3.0)
    assert b[0] == 0.2 and abs(b[-1] - 3.0) < 1e-12 and np.allclose(b[1:] / b[:-1], (15.0) ** (1 / 31))
    g = linear_gamma(1000)
    assert g[0] == 3.0 and abs(g[-1] - 0.01) < 1e-12 and np.allclose(np.diff(g), (0.01 - 3.0) / 999)
    assert list(linear_gamma(1)) == [3.0]
    s = mixed_sizes(256)
    assert s.count(6) == 52 and all(s.count(L) == 51 for L in (8, 10, 12, 15))
