"""Pins of the nonlocal kernel surrogate's oracle (Sec. 6, Eqs. 6.5-6.6):
the Bernstein basis, the operator on constant fields and on Fourier modes
(closed-form multiplier), recovery of a planted kernel from data generated
by an independent FFT convolution, and Adam against the closed-form
Tikhonov minimiser."""
import numpy as np
import pytest

from oracle import nonlocal_oracle as N


def test_bernstein_basis():
    t = np.linspace(0.0, 1.0, 11)
    for M in (0, 1, 3, 6):
        B = N.bernstein(M, t)
        np.testing.assert_allclose(B.sum(axis=0), 1.0, rtol=0, atol=1e-15)     # partition of unity
        assert (B >= 0.0).all()
        assert B[0, 0] == 1.0 and B[M, -1] == 1.0
    # degree 2 by hand at t = 1/4: (9/16, 6/16, 1/16)
    np.testing.assert_allclose(N.bernstein(2, 0.25), [9 / 16, 6 / 16, 1 / 16], rtol=0, atol=1e-16)


def test_operator_vanishes_on_constants():
    u = np.ones((3, 6, 8, 10)) * np.array([1.5, -2.0, 0.25])[:, None, None, None]
    out = N.apply_operator([0.3, -1.0, 2.0, 0.7], u, 2.6)
    assert np.abs(out).max() < 1e-13


@pytest.mark.parametrize("shape,k", [((16, 12), (3, -2)), ((8, 10, 12), (1, 2, -3))])
def test_operator_on_a_fourier_mode(shape, k):
    """u = cos(xi . x): L[u] = m(xi) u with m = sum over offsets inside the
    horizon of K(|r|) (cos(xi . r) - 1), the offsets enumerated here by a
    brute-force scan of the periodic grid's minimum images."""
    d = len(shape)
    delta = 3.2
    c = np.array([0.4, -0.3, 1.1, 0.2])
    xi = np.array([2 * np.pi * k[a] / shape[a] for a in range(d)])
    pos = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    phase = sum(xi[a] * pos[a] for a in range(d))
    u = np.stack([np.cos(phase), 0.5 * np.cos(phase)])
    mult = 0.0
    for idx in np.ndindex(*shape):
        r = np.array([v if v <= n // 2 else v - n for v, n in zip(idx, shape)], dtype=np.float64)
        rho = np.sqrt(r @ r)
        if 0.0 < rho < delta:
            t = rho / delta
            K = sum(c[m] * N.comb(3, m) * t ** m * (1 - t) ** (3 - m) for m in range(4))
            mult += K * (np.cos(xi @ r) - 1.0)
    np.testing.assert_allclose(N.apply_operator(c, u, delta), mult * u, rtol=0, atol=1e-12)


def kernel_image(c, shape, delta):
    """K_c(|r|) on the periodic grid at the minimum-image offsets (origin 0)."""
    d = len(shape)
    M = len(c) - 1
    img = np.zeros(shape)
    for idx in np.ndindex(*shape):
        r = np.array([v if v <= n // 2 else v - n for v, n in zip(idx, shape)], dtype=np.float64)
        rho = np.sqrt(r @ r)
        if 0.0 < rho < delta:
            img[idx] = float(np.dot(c, N.bernstein(M, rho / delta)))
    return img


def operator_by_fft(c, u, delta):
    """L_c[u] = (K * u)(x) - (sum K) u(x), the convolution by FFT."""
    shape = u.shape[1:]
    img = kernel_image(c, shape, delta)
    axes = tuple(range(1, u.ndim))
    # sum_r K(r) u(x + r) = correlation; K is even, so it equals the convolution
    conv = np.fft.ifftn(np.fft.fftn(u, axes=axes) * np.fft.fftn(img)[None], axes=axes).real
    return conv - img.sum() * u


def test_planted_kernel_is_recovered():
    rng = np.random.default_rng(4)
    shape, delta, c_true = (10, 12, 14), 3.5, np.array([0.8, -0.4, 0.25, 1.3, -0.6])
    us = [rng.normal(size=(3,) + shape) for _ in range(3)]
    gammas = [operator_by_fft(c_true, u, delta) for u in us]
    G, g, gg = N.normal_equations(us, gammas, len(c_true) - 1, delta)
    c = N.fit_closed(G, g, 0.0)
    np.testing.assert_allclose(c, c_true, rtol=0, atol=1e-9)
    assert N.loss(c, G, g, gg, 0.0) < 1e-12 * gg     # the expanded quadratic cancels to rounding
    # the operator itself agrees with the FFT route
    np.testing.assert_allclose(N.apply_operator(c_true, us[0], delta), gammas[0], rtol=0,
                               atol=1e-12 * np.abs(gammas[0]).max())


def test_adam_reaches_the_tikhonov_minimiser():
    rng = np.random.default_rng(6)
    shape, delta, M, lam = (8, 8, 8), 2.8, 3, 0.05
    us = [rng.normal(size=(3,) + shape) for _ in range(2)]
    gammas = [rng.normal(size=(3,) + shape) for _ in range(2)]
    G, g, gg = N.normal_equations(us, gammas, M, delta)
    scale = np.trace(G) / (M + 1)
    Gs, gs, lams = G / scale, g / scale, lam / scale        # same minimiser, unit-scale curvature
    c_star = N.fit_closed(Gs, gs, lams)
    np.testing.assert_allclose(c_star, N.fit_closed(G, g, lam), rtol=1e-9)
    c = N.fit_adam(Gs, gs, lams, steps=50000, lr=1e-3)
    np.testing.assert_allclose(c, c_star, rtol=0, atol=1e-6 * np.abs(c_star).max())
    assert N.loss(c, G, g, gg, lam) <= N.loss(c_star, G, g, gg, lam) * (1 + 1e-9)


# ------------------------------------------------- isotropic matrix kernel (form 1)
def kernel_pair(c, rho, delta):
    """(K1, K2) at distance rho for coefficients (c1_0..c1_M, c2_0..c2_M)."""
    c = np.asarray(c, dtype=np.float64)
    M = len(c) // 2 - 1
    t = rho / delta
    b = [N.comb(M, m) * t ** m * (1 - t) ** (M - m) for m in range(M + 1)]
    return float(np.dot(c[:M + 1], b)), float(np.dot(c[M + 1:], b))


def min_image_offsets(shape):
    """Every grid offset as its minimum-image vector in component order (x
    first), with its array index."""
    for idx in np.ndindex(*shape):
        r_arr = [v if v <= n // 2 else v - n for v, n in zip(idx, shape)]
        yield idx, np.array(r_arr[::-1], dtype=np.float64)


@pytest.mark.parametrize("shape,k", [((16, 12), (3, -2)), ((8, 10, 12), (1, 2, -3))])
def test_matrix_kernel_on_a_fourier_mode(shape, k):
    """u_a = v_a cos(xi . x): L[u] = M(xi) v cos(xi . x) with
    M = sum_r (cos(xi . r) - 1)(K1 I + K2 e e^T), the offsets enumerated by
    a scan of the grid's minimum images, directions in component order."""
    d = len(shape)
    delta = 3.2
    c = np.array([0.4, -0.3, 1.1, 0.2, -0.7, 0.5, 0.9, -0.2])
    v = np.array([1.0, 0.5, -0.3][:d])
    xi_arr = np.array([2 * np.pi * k[a] / shape[a] for a in range(d)])     # array order
    pos = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    phase = sum(xi_arr[a] * pos[a] for a in range(d))
    u = v.reshape((d,) + (1,) * d) * np.cos(phase)
    Mx = np.zeros((d, d))
    for idx, r in min_image_offsets(shape):
        rho = np.sqrt(r @ r)
        if 0.0 < rho < delta:
            K1, K2 = kernel_pair(c, rho, delta)
            e = r / rho
            xr = sum(xi_arr[a] * idx_r for a, idx_r in enumerate(r[::-1]))    # xi . r in array order
            Mx += (np.cos(xr) - 1.0) * (K1 * np.eye(d) + K2 * np.outer(e, e))
    want = (Mx @ v).reshape((d,) + (1,) * d) * np.cos(phase)
    np.testing.assert_allclose(N.apply_operator(c, u, delta, form=1), want, rtol=0, atol=1e-12)


def matrix_operator_by_fft(c, u, delta):
    """out_a = sum_b (K_ab * u_b) - (sum_r K_ab(r)) u_b with the 3x3 kernel
    image on the periodic grid, by FFT."""
    shape = u.shape[1:]
    d = len(shape)
    img = np.zeros((d, d) + shape)
    for idx, r in min_image_offsets(shape):
        rho = np.sqrt(r @ r)
        if 0.0 < rho < delta:
            K1, K2 = kernel_pair(c, rho, delta)
            e = r / rho
            img[(slice(None), slice(None)) + idx] = K1 * np.eye(d) + K2 * np.outer(e, e)
    axes = tuple(range(1, d + 1))
    uh = np.fft.fftn(u, axes=axes)
    kh = np.fft.fftn(img, axes=tuple(range(2, d + 2)))
    conv = np.fft.ifftn(np.einsum("ab...,b...->a...", kh, uh), axes=axes).real
    tot = img.sum(axis=tuple(range(2, d + 2)))
    return conv - np.einsum("ab,b...->a...", tot, u)


@pytest.mark.parametrize("shape", [(10, 12, 14), (20, 18)])
def test_planted_matrix_kernel_is_recovered(shape):
    rng = np.random.default_rng(8)
    d = len(shape)
    delta = 3.5
    c_true = np.array([0.8, -0.4, 0.25, 1.3, 0.6, -0.9, 0.3, 0.45])
    us = [rng.normal(size=(d,) + shape) for _ in range(3)]
    gammas = [matrix_operator_by_fft(c_true, u, delta) for u in us]
    np.testing.assert_allclose(N.apply_operator(c_true, us[0], delta, form=1), gammas[0], rtol=0,
                               atol=1e-12 * np.abs(gammas[0]).max())
    G, g, gg = N.normal_equations(us, gammas, 3, delta, form=1)
    c = N.fit_closed(G, g, 0.0)
    np.testing.assert_allclose(c, c_true, rtol=0, atol=1e-8)


def test_matrix_operator_is_self_adjoint_and_kills_constants():
    rng = np.random.default_rng(9)
    shape, delta = (8, 9, 10), 2.9
    c = rng.normal(size=6)
    u, v = rng.normal(size=(3,) + shape), rng.normal(size=(3,) + shape)
    lu, lv = N.apply_operator(c, u, delta, form=1), N.apply_operator(c, v, delta, form=1)
    assert abs(np.sum(v * lu) - np.sum(u * lv)) < 1e-11 * np.abs(lu).max() * np.abs(v).sum()
    const = np.ones((3,) + shape) * np.array([0.3, -1.2, 2.0])[:, None, None, None]
    assert np.abs(N.apply_operator(c, const, delta, form=1)).max() < 1e-13


def test_long_wave_stiffness_matches_the_small_wavenumber_multiplier():
    """The product's long-wavelength stiffness of a matrix-kernel operator
    against the exact Fourier multiplier sum_r (K1 I + K2 e e^T)(cos xi.r - 1)
    at a small wavevector: M(xi) v = -(C grad grad) v, i.e.
    M_ab = -(C11 - C44 or C44 ... ) assembled from (C11, C12, C44), to the
    fourth-order truncation error."""
    from paper_2601_00822_amd.nonlocal_operator import NonlocalOperator
    rng = np.random.default_rng(17)
    delta, M = 4.5, 5
    c = rng.normal(size=2 * (M + 1))
    C11, C12, C44 = NonlocalOperator(c, delta, form=1).long_wave_stiffness()
    xi = np.array([0.7, -1.1, 0.4]) * 1e-3
    Mx = np.zeros((3, 3))
    R = int(np.ceil(delta))
    for idx in np.ndindex(2 * R + 1, 2 * R + 1, 2 * R + 1):
        r = np.array(idx, dtype=np.float64) - R                 # component order (x first)
        rho = np.sqrt(r @ r)
        if 0.0 < rho < delta:
            K1, K2 = kernel_pair(c, rho, delta)
            e = r / rho
            Mx += (np.cos(xi @ r) - 1.0) * (K1 * np.eye(3) + K2 * np.outer(e, e))
    # div(C grad) of a plane wave: -(C_aibj xi_i xi_j) for a cubic C
    want = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            if a == b:
                want[a, a] = -(C11 * xi[a] ** 2 + C44 * (xi @ xi - xi[a] ** 2))
            else:
                want[a, b] = -(C12 + C44) * xi[a] * xi[b]
    np.testing.assert_allclose(Mx, want, rtol=0, atol=1e-5 * np.abs(want).max())
