"""Host-only checks of the seeded input generators shared by both paths."""
import numpy as np
import pytest

import gen


@pytest.mark.parametrize("cell,vf,rmin,rmax", [(16, 0.2, 3.0, 6.0), (16, 0.3, 3.0, 6.0),
                                               (8, 0.2, 1.5, 2.5), (16, 0.1, 3.0, 6.0)])
def test_rsa_cell_terminates_near_target(cell, vf, rmin, rmax):
    # a rejection after the overshoot test must not reset the failure count,
    # otherwise the loop never gives up on a saturated cell
    ph, got = gen.rsa_cell(cell, 3, vf, rmin, rmax, seed=7)
    assert ph.shape == (cell,) * 3 and ph.dtype == np.uint8
    assert abs(got - ph.mean()) < 1e-12
    assert vf - 0.02 <= got <= vf + 0.1


def test_rsa_cell_is_seeded():
    a, _ = gen.rsa_cell(16, 3, 0.2, 3.0, 6.0, seed=3)
    b, _ = gen.rsa_cell(16, 3, 0.2, 3.0, 6.0, seed=3)
    c, _ = gen.rsa_cell(16, 3, 0.2, 3.0, 6.0, seed=4)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_dipole_force_sums_to_zero():
    f = gen.dipole_force((16, 32), (8.0, 16.0), 5.0, (0.6, 0.8), sep=4)
    assert np.abs(f.sum(axis=(1, 2))).max() < 1e-13


def test_bump_force_support_and_peak():
    f = gen.bump_force((32, 32), (16.0, 16.0), 6.0, (1.0, 0.0))
    assert abs(f[0].max() - np.exp(-1.0)) < 1e-15
    pos = gen.grid_positions((32, 32))
    r2 = (pos[0] - 16.0) ** 2 + (pos[1] - 16.0) ** 2
    assert np.all(f[0][r2 >= 36.0] == 0.0) and np.all(f[1] == 0.0)


def test_shift_sets():
    s = gen.all_shifts(4, 3)
    assert s.shape == (64, 3) and len({tuple(r) for r in s}) == 64
    t = gen.sample_shifts(4, 3, 10, seed=1)
    assert t.shape == (10, 3) and len({tuple(r) for r in t}) == 10
    assert set(map(tuple, t)) <= set(map(tuple, s))


def test_inclusion_per_cell_fraction():
    ph, vf = gen.inclusion_per_cell((32, 32, 32), 16, 0.2)
    assert abs(vf - 0.2) < 0.02 and abs(ph.mean() - vf) < 1e-12


def test_point_force():
    f = gen.point_force((4, 6, 8), 1)
    assert f.shape == (3, 4, 6, 8) and f.sum() == 1.0 and f[1, 0, 0, 0] == 1.0
