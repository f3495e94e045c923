"""Pins of the oracle's deterministic-structure average (Sec. 3, Eq. 3.8)."""
import numpy as np

import gen
from oracle import lsfft_oracle as O

LAME = O.lame_from_young(gen.Material.two_phase(1.0, 10.0).table())


def _maps(shape, seeds):
    return [(np.random.default_rng(s).random(shape) < 0.35).astype(np.uint8) for s in seeds]


def test_identical_realisations_reduce_to_one_solve():
    shape = (12, 16)
    ph = _maps(shape, [3])[0]
    f = np.random.default_rng(4).normal(size=(2,) + shape)
    avg, iters = O.realization_average([ph, ph, ph], LAME, f, tol=1e-10)
    res = O.solve_basic(ph, LAME, f, tol=1e-10)
    assert iters == [res.iters] * 3
    np.testing.assert_allclose(avg[4:7], O.to_voigt(res.eps), rtol=0, atol=1e-13 * np.abs(res.eps).max())
    np.testing.assert_allclose(avg[0:2], res.u, rtol=0, atol=1e-13 * np.abs(res.u).max())
    np.testing.assert_array_equal(avg[-1], (ph == 1).astype(float))


def test_shifted_copies_equal_the_translated_average():
    # a rigidly shifted microstructure (Eq. 3.3, phase_chi(x) = phase(x - chi))
    # is one realisation: averaging the shifted copies is the translated average
    shape = (8, 8, 8)
    ph = _maps(shape, [5])[0]
    f = gen.bump_force(shape, (3.2, 4.1, 2.7), 3.0, gen.random_direction(3, 6))
    shifts = np.array([[0, 0, 0], [1, 2, 3], [4, 0, 7]])
    reals = [np.roll(ph, shift=tuple(int(c) for c in chi), axis=(0, 1, 2)) for chi in shifts]
    a, _ = O.realization_average(reals, LAME, f, tol=1e-10)
    b, _ = O.translate_average(ph, LAME, f, shifts, tol=1e-10)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-14 * np.abs(b).max())


def test_occupancy_is_the_mean_indicator_and_linear_in_force():
    shape = (16, 12)
    maps = _maps(shape, [7, 8, 9, 10])
    f = np.random.default_rng(11).normal(size=(2,) + shape)
    a, _ = O.realization_average(maps, LAME, f, tol=1e-11)
    b, _ = O.realization_average(maps, LAME, -2.5 * f, tol=1e-11)
    np.testing.assert_allclose(a[-1], np.mean([(m == 1) for m in maps], axis=0))
    np.testing.assert_allclose(b[:-1], -2.5 * a[:-1], rtol=0, atol=1e-9 * np.abs(a[:-1]).max())
