"""Pins of the oracle's Krylov and accelerated schemes (Sec. 5): Algorithm 3
(plain conjugate gradients on the displacement fluctuation, Eqs. 5.17-5.22)
and Anderson acceleration of the basic scheme.

The references here are built from the dense real-space operators of
``oracle/dense.py`` (assembled from the DFT definition, no FFT routine, no
spectral operator of the iterative oracle):

* every scheme reaches the minimum-norm dense solve of the same discrete
  system (Eq. 5.5), whatever its start;
* conjugate gradients: iterate k minimizes the energy norm of the error over
  the start plus the Krylov space K_k(A, r_0) -- the defining property of CG,
  checked by a projected dense solve;
* Anderson acceleration with memory m and mixing 1 on a linear map
  g(x) = x + N0 (P f - A x): for k <= m its iterate k + 1 is g applied to the
  k-th GMRES iterate of (N0 A) x = N0 P f from the same start (Walker & Ni,
  SIAM J. Numer. Anal. 49 (2011), Theorem 2.2), GMRES computed here by a
  dense least-squares solve over an explicit Krylov basis; N0 is the
  pseudo-inverse of the dense reference-medium operator.
"""
import numpy as np
import pytest

import gen
from oracle import dense
from oracle import lsfft_oracle as O

LAME = O.lame_from_young(gen.Material.two_phase(1.0, 100.0).table())


def problem(shape, seed):
    rng = np.random.default_rng(seed)
    ph = (rng.random(shape) < 0.35).astype(np.uint8)
    f = rng.normal(size=(len(shape),) + shape)
    return ph, f


def flat(u):
    return np.asarray(u).reshape(-1)


@pytest.mark.parametrize("shape", [(8, 8), (4, 4, 4)])
def test_alg3_and_anderson_reach_the_dense_solution(shape):
    ph, f = problem(shape, 3)
    u, e, s = dense.dense_solve(ph, LAME, f)
    for res in (O.solve_cg_alg3(ph, LAME, f, tol=1e-12),
                O.solve_cg_alg3(ph, LAME, f, tol=1e-12, start="zero"),
                O.solve_anderson(ph, LAME, f, tol=1e-12, m=5),
                O.solve_anderson(ph, LAME, f, tol=1e-12, m=1)):
        assert res.status == 0
        assert O.relative_strain_error(res.eps, e) < 1e-10
        assert np.abs(res.u - u).max() < 1e-9 * np.abs(u).max()


def test_alg3_printed_and_zero_starts_differ_in_iterates_not_in_the_limit():
    ph, f = problem((8, 8), 4)
    a = O.solve_cg_alg3(ph, LAME, f, tol=1e-30, max_iter=0)
    b = O.solve_cg_alg3(ph, LAME, f, tol=1e-30, max_iter=0, start="zero")
    ref = O.solve_basic(ph, LAME, f, tol=1e-30, max_iter=0)
    # the zero start is the free term u^b; the printed one adds b^A
    np.testing.assert_allclose(b.u, ref.u, rtol=0, atol=1e-13 * np.abs(ref.u).max())
    assert np.abs(a.u - b.u).max() > 1e-3 * np.abs(b.u).max()


@pytest.mark.parametrize("start", ["printed", "zero"])
@pytest.mark.parametrize("shape", [(8, 8), (4, 4, 4)])
def test_alg3_iterates_minimize_the_energy_error_over_krylov_spaces(shape, start):
    ph, f = problem(shape, 5)
    d = len(shape)
    A, _ = dense.assemble(ph, LAME)
    P = dense.zero_mode_projector(shape)
    pf = np.concatenate([P @ flat(f[c]) for c in range(d)])
    x0 = flat(O.solve_cg_alg3(ph, LAME, f, tol=1e-30, max_iter=0, start=start).u)
    r0 = pf - A @ x0
    for k in range(1, 6):
        cols = [r0]
        for _ in range(k - 1):
            cols.append(A @ cols[-1])
        V, _ = np.linalg.qr(np.stack(cols, axis=1))
        y = np.linalg.solve(V.T @ A @ V, V.T @ r0)
        xk = x0 + V @ y
        got = flat(O.solve_cg_alg3(ph, LAME, f, tol=1e-30, max_iter=k, start=start).u)
        assert np.abs(got - xk).max() < 1e-9 * np.abs(xk).max(), k


def test_anderson_without_memory_is_the_basic_scheme():
    ph, f = problem((8, 8), 6)
    for k in (0, 1, 2, 7):
        a = O.solve_anderson(ph, LAME, f, tol=1e-30, max_iter=k, m=0)
        b = O.solve_displacement_update(ph, LAME, f, tol=1e-30, max_iter=k)
        np.testing.assert_allclose(a.u, b.u, rtol=0, atol=1e-14 * np.abs(b.u).max())
        assert a.history == b.history


@pytest.mark.parametrize("shape", [(8, 8), (4, 4, 4)])
def test_anderson_is_g_of_gmres_on_the_linear_map(shape):
    ph, f = problem(shape, 7)
    d = len(shape)
    lam0, mu0 = O.reference_medium(LAME)
    A, _ = dense.assemble(ph, LAME)
    K0, _ = dense.assemble(np.zeros(shape, dtype=np.uint8), np.array([[lam0, mu0]]))
    N0 = np.linalg.pinv(K0, rcond=1e-12, hermitian=True)
    P = dense.zero_mode_projector(shape)
    pf = np.concatenate([P @ flat(f[c]) for c in range(d)])
    B = N0 @ A                                  # (I - G) of the map g(x) = x + N0 (P f - A x)
    c = N0 @ pf

    def g(x):
        return x + N0 @ (pf - A @ x)

    m = 5
    x0 = flat(O.solve_anderson(ph, LAME, f, tol=1e-30, max_iter=0, m=m).u)
    f0 = c - B @ x0
    for k in range(1, m + 1):
        cols = [f0]
        for _ in range(k - 1):
            cols.append(B @ cols[-1])
        K = np.stack(cols, axis=1)
        y = np.linalg.lstsq(B @ K, f0, rcond=None)[0]
        x_gmres = x0 + K @ y
        want = g(x_gmres)
        got = flat(O.solve_anderson(ph, LAME, f, tol=1e-30, max_iter=k + 1, m=m).u)
        assert np.abs(got - want).max() < 1e-8 * np.abs(want).max(), k


@pytest.mark.parametrize("m", [1, 2])
def test_anderson_window_holds_the_last_m_steps(m):
    """Past the first m steps the memory is a sliding window: iterate k + 1
    is the affine combination sum_i a_i g(x_i) of the last m + 1 iterates
    with sum_i a_i = 1 that minimizes ||sum_i a_i (g(x_i) - x_i)|| (the
    constrained form of the method, Walker & Ni eq. 1.2), evaluated with the
    dense operators on the oracle's own iterates."""
    shape = (8, 8)
    ph, f = problem(shape, 8)
    d = len(shape)
    lam0, mu0 = O.reference_medium(LAME)
    A, _ = dense.assemble(ph, LAME)
    K0, _ = dense.assemble(np.zeros(shape, dtype=np.uint8), np.array([[lam0, mu0]]))
    N0 = np.linalg.pinv(K0, rcond=1e-12, hermitian=True)
    P = dense.zero_mode_projector(shape)
    pf = np.concatenate([P @ flat(f[c]) for c in range(d)])

    def resid(x):
        return N0 @ (pf - A @ x)

    xs = [flat(O.solve_anderson(ph, LAME, f, tol=1e-30, max_iter=j, m=m).u) for j in range(m + 5)]
    for k in range(m, m + 4):
        win = xs[k - m:k + 1]
        Fm = np.stack([resid(x) for x in win], axis=1)
        # minimize |Fm a| with sum a = 1: a = a_last-eliminated least squares
        base = Fm[:, -1]
        Dm = Fm[:, :-1] - base[:, None]
        c = np.linalg.lstsq(Dm, -base, rcond=None)[0]
        a = np.concatenate([c, [1.0 - c.sum()]])
        want = sum(ai * (x + resid(x)) for ai, x in zip(a, win))
        assert np.abs(xs[k + 1] - want).max() < 1e-8 * np.abs(want).max(), k
