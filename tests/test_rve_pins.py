"""Pins of the oracle's RVE identification (Definition 2.2): radial maxima
against brute force over periodic images, the tensor magnitude against the
full tensor's Frobenius norm, and the RVE radius of fields with a known
decay."""
import itertools

import numpy as np

from oracle import lsfft_oracle as O


def _brute_radial(field, center, h, dr):
    shape = field.shape
    d = len(shape)
    half = np.sqrt(sum((0.5 * shape[a] * h[a]) ** 2 for a in range(d)))
    nb = int(np.floor(half / dr)) + 1
    out = np.zeros(nb)
    for idx in itertools.product(*[range(n) for n in shape]):
        best = np.inf
        for img in itertools.product((-1, 0, 1), repeat=d):      # nearest periodic image of the centre
            r2 = sum(((idx[a] - center[a] - img[a] * shape[a]) * h[a]) ** 2 for a in range(d))
            best = min(best, r2)
        b = min(int(np.sqrt(best) // dr), nb - 1)
        out[b] = max(out[b], field[idx])
    return out


def test_radial_maxima_against_brute_force():
    rng = np.random.default_rng(3)
    for shape, center, h, dr in [((12, 10), (2.5, 8.0), (1.0, 1.0), 1.0),
                                 ((6, 8, 10), (5.2, 0.0, 9.5), (1.0, 0.5, 2.0), 0.75)]:
        field = rng.random(shape)
        got = O.radial_maxima(field, center, h, dr)
        want = _brute_radial(field, center, h, dr)
        np.testing.assert_allclose(got, want, rtol=0, atol=0)


def test_tensor_magnitude_is_the_frobenius_norm():
    rng = np.random.default_rng(4)
    for d, s in ((2, 3), (3, 6)):
        tv = rng.normal(size=(s, 5, 7))
        full = np.zeros((d, d, 5, 7))
        for c, (a, b) in enumerate(O.VOIGT[d]):
            full[a, b] = tv[c]
            full[b, a] = tv[c]
        want = np.sqrt((full ** 2).sum(axis=(0, 1)))
        np.testing.assert_allclose(O.tensor_magnitude(tv), want, rtol=1e-15)


def _gauss_avg(shape, center, width):
    d = len(shape)
    s = 6 if d == 3 else 3
    grids = np.meshgrid(*[np.arange(n, dtype=float) for n in shape], indexing="ij")
    r2 = sum((grids[a] - center[a]) ** 2 for a in range(d))
    g = np.exp(-r2 / (2 * width ** 2))
    avg = np.zeros((2 * d + 4 * s + 1,) + shape)
    avg[2 * d] = g                    # eps_11
    avg[2 * d + 2 * s + 1] = 3.0 * g  # sigma_22
    return avg, np.sqrt(r2), g


def test_rve_radius_of_a_gaussian():
    shape, center, width, tol = (40, 40), (20.0, 20.0), 2.5, 1e-3
    avg, r, g = _gauss_avg(shape, center, width)
    radius, fits, pe, ps = O.rve_radius(avg, center, support_radius=6.0, tol=tol)
    # the RVE starts at the first bin beyond every voxel with g >= tol max g
    want = np.floor(r[g >= tol * g.max()].max()) + 1
    assert radius == want
    # analytic: the level set g = tol sits at width sqrt(2 ln(1/tol))
    assert abs(radius - width * np.sqrt(2 * np.log(1 / tol))) <= 1.0 + 1e-12
    assert fits == (radius + 3.0 <= 20.0)
    np.testing.assert_allclose(ps, 3.0 * pe)


def test_minimum_image_and_enlargement_flag():
    shape = (32, 32)
    avg, _, _ = _gauss_avg(shape, (0.0, 0.0), 1.5)
    # the field peaks at the corner voxel; with the centre at the opposite
    # corner the nearest image is one diagonal step away
    radius, _, _, _ = O.rve_radius(avg, (31.0, 31.0), 0.0, 1e-3)
    radius0, _, _, _ = O.rve_radius(avg, (0.0, 0.0), 0.0, 1e-3)
    assert radius0 < radius <= radius0 + 2
    r_small, fits_small, _, _ = O.rve_radius(avg, (0.0, 0.0), 10.0, 1e-3)
    r_big, fits_big, _, _ = O.rve_radius(avg, (0.0, 0.0), 30.0, 1e-3)
    assert fits_small and not fits_big and r_small == r_big
