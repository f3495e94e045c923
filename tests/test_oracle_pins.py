"""Pins of the FP64 oracle against things other than itself.

Each test fixes part of the oracle by a closed form, an identity of the
paper, a brute-force computation or an invariant, chosen so that a dropped
term, a wrong sign, a wrong index or a transposed operand in the oracle fails
at least one of them.  CPU only.
"""
import numpy as np
import pytest

import gen
from oracle import dense
from oracle import lsfft_oracle as O

MAT10 = gen.Material.two_phase(1.0, 10.0)
LAME10 = O.lame_from_young(MAT10.table())


def rand_phase(shape, seed, p=0.35):
    return (np.random.default_rng(seed).random(shape) < p).astype(np.uint8)


def rand_force(shape, seed):
    return np.random.default_rng(seed).normal(size=(len(shape),) + tuple(shape))


# ---------------------------------------------------------------- materials

def test_lame_pin_bulk_modulus_identity():
    """lambda + 2 mu / 3 equals the bulk modulus E / (3 (1 - 2 nu)), and
    mu = E / (2 (1 + nu)): the matrix phase E = 1, nu = 0.3 gives
    (0.576923..., 0.384615...)."""
    tab = np.array([[1.0, 0.3], [10.0, 0.3], [3.0, 0.1], [2.0, 0.45]])
    lame = O.lame_from_young(tab)
    k = tab[:, 0] / (3.0 * (1.0 - 2.0 * tab[:, 1]))
    np.testing.assert_allclose(lame[:, 0] + 2.0 * lame[:, 1] / 3.0, k, rtol=1e-14)
    np.testing.assert_allclose(lame[0], [15.0 / 26.0, 10.0 / 26.0], rtol=1e-14)


def test_reference_medium_mean_of_extremes():
    lame = np.array([[1.0, 2.0], [5.0, 0.5], [3.0, 1.0]])
    assert O.reference_medium(lame) == (3.0, 1.25)


# ---------------------------------------------------------------- DFT (P10)

@pytest.mark.parametrize("shape", [(6,), (8,), (4, 6), (6, 4, 8)])
def test_fft_matches_bruteforce_dft(shape):
    """numpy's transform used by the oracle equals the O(N^2) sums of
    Eqs. 4.3-4.5 (forward, unnormalised, exp(-i...)) and the inverse Eq. 4.4."""
    rng = np.random.default_rng(0)
    a = rng.normal(size=shape)
    d = len(shape)
    idx = np.stack(np.meshgrid(*[np.arange(n) for n in shape], indexing="ij"), -1).reshape(-1, d)
    ph = np.zeros((len(idx), len(idx)))
    for ax, n in enumerate(shape):
        ph += np.outer(idx[:, ax], idx[:, ax]) / n
    F = np.exp(-2j * np.pi * ph)
    full = (F @ a.ravel()).reshape(shape)
    got = O.fft_r(a[None], shape)[0]
    np.testing.assert_allclose(got, full[..., : shape[-1] // 2 + 1], atol=1e-12)
    back = (np.conj(F) @ full.ravel()).reshape(shape).real / len(idx)
    np.testing.assert_allclose(back, a, atol=1e-12)
    np.testing.assert_allclose(O.ifft_r(got[None], shape)[0], a, atol=1e-12)


def test_wavevector_derivative_of_trig_polynomial():
    """i xi f^ differentiates a band-limited periodic field exactly (Eq. 4.8)
    and the Nyquist wavevector is zero."""
    shape = (8, 12)
    y, x = np.meshgrid(np.arange(8), np.arange(12), indexing="ij")
    f = np.sin(2 * np.pi * 3 * x / 12) * np.cos(2 * np.pi * 2 * y / 8)
    dfdx = (2 * np.pi * 3 / 12) * np.cos(2 * np.pi * 3 * x / 12) * np.cos(2 * np.pi * 2 * y / 8)
    dfdy = -(2 * np.pi * 2 / 8) * np.sin(2 * np.pi * 3 * x / 12) * np.sin(2 * np.pi * 2 * y / 8)
    xi = O.wavevectors(shape)
    fh = O.fft_r(f[None], shape)[0]
    np.testing.assert_allclose(O.ifft_r((1j * xi[0] * fh)[None], shape)[0], dfdx, atol=1e-12)
    np.testing.assert_allclose(O.ifft_r((1j * xi[1] * fh)[None], shape)[0], dfdy, atol=1e-12)
    assert xi[0].ravel()[-1] == 0.0 and xi[1].ravel()[4] == 0.0
    z = O.zero_set(shape)
    assert z.sum() == 4 and z[0, 0] and z[4, 0] and z[0, -1] and z[4, -1]


# ---------------------------------------------------------------- Green operators (P1, P2)

def explicit_U0(z, lam0, mu0):
    """Eqs. 2.16-2.18 written out: U0 = U1 / (4 mu0) + c U2 with
    U1_ijkl = -|z|^-2 (d_ki z_l z_j + d_li z_k z_j + d_kj z_l z_i + d_lj z_k z_i)
    and U2_ijkl = |z|^-4 z_i z_j z_k z_l (index h of the print read as l)."""
    d = z.size
    n2 = z @ z
    I = np.eye(d)
    U1 = -(np.einsum("ki,l,j->ijkl", I, z, z) + np.einsum("li,k,j->ijkl", I, z, z)
           + np.einsum("kj,l,i->ijkl", I, z, z) + np.einsum("lj,k,i->ijkl", I, z, z)) / n2
    U2 = np.einsum("i,j,k,l->ijkl", z, z, z, z) / n2 ** 2
    return U1 / (4 * mu0) + (lam0 + mu0) / (mu0 * (lam0 + 2 * mu0)) * U2


@pytest.mark.parametrize("d", [2, 3])
def test_U0_matches_paper_tensor(d):
    """The oracle's U0 (through N0, divergence and symmetric gradient)
    equals the explicit tensor of Eqs. 2.16-2.18 on random wavevectors."""
    rng = np.random.default_rng(d)
    lam0, mu0 = 1.7, 0.9
    for _ in range(5):
        z = rng.normal(size=d)
        xi = [np.array([z[a]]) for a in range(d)]
        tau = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
        tau = 0.5 * (tau + tau.T)
        got = O.apply_U0(tau[..., None], xi, lam0, mu0)[..., 0]
        want = np.einsum("ijkl,kl->ij", explicit_U0(z, lam0, mu0), tau)
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("d", [2, 3])
def test_gamma0_projector_identities(d):
    """Gamma0 = -U0: Gamma0 L0 Gamma0 = Gamma0 and Gamma0 L0 sym(xi (x) v) = sym(xi (x) v)."""
    rng = np.random.default_rng(10 + d)
    lam0, mu0 = 2.3, 0.7
    I = np.eye(d)
    L0 = (lam0 * np.einsum("ij,kl->ijkl", I, I)
          + mu0 * (np.einsum("ik,jl->ijkl", I, I) + np.einsum("il,jk->ijkl", I, I)))
    for _ in range(4):
        z = rng.normal(size=d)
        G = -explicit_U0(z, lam0, mu0)
        GLG = np.einsum("ijab,abcd,cdkl->ijkl", G, L0, G)
        np.testing.assert_allclose(GLG, G, atol=1e-12)
        v = rng.normal(size=d)
        e = 0.5 * (np.outer(z, v) + np.outer(v, z))
        np.testing.assert_allclose(np.einsum("ijab,abcd,cd->ij", G, L0, e), e, atol=1e-12)


def test_N0_is_inverse_acoustic_tensor_P_S_split():
    """N0 equals the longitudinal/transverse split n n / ((lam+2mu)|xi|^2) +
    (I - n n) / (mu |xi|^2) and inverts K0 = mu |xi|^2 I + (lam+mu) xi xi^T."""
    rng = np.random.default_rng(3)
    lam0, mu0 = 0.8, 1.9
    for d in (2, 3):
        z = rng.normal(size=d)
        n = z / np.linalg.norm(z)
        k2 = z @ z
        want = np.outer(n, n) / ((lam0 + 2 * mu0) * k2) + (np.eye(d) - np.outer(n, n)) / (mu0 * k2)
        xi = [np.array([z[a]]) for a in range(d)]
        got = np.stack([O.apply_N0(np.eye(d)[:, c][:, None].astype(complex), xi, lam0, mu0)[:, 0]
                        for c in range(d)], axis=1).real
        np.testing.assert_allclose(got, want, rtol=1e-13)
        K0 = mu0 * k2 * np.eye(d) + (lam0 + mu0) * np.outer(z, z)
        np.testing.assert_allclose(K0 @ got, np.eye(d), atol=1e-13)


def test_U0_vanishes_at_origin():
    """(U0 * tau)(0) = 0 for any field (stated after Eq. 2.18)."""
    shape = (8, 6)
    tau = np.random.default_rng(0).normal(size=(2, 2) + shape)
    tau = 0.5 * (tau + tau.transpose(1, 0, 2, 3))
    out = O.apply_U0(O.fft_r(tau, shape), O.wavevectors(shape), 1.0, 1.0)
    assert np.abs(out[..., 0, 0]).max() == 0.0


@pytest.mark.parametrize("d", [2, 3])
def test_eq_2_27_identity(d):
    """U0 * (L0 eps) = <eps> - eps for compatible eps = E + sym grad u (Eq. 2.27)."""
    shape = (8, 10) if d == 2 else (6, 8, 4)
    rng = np.random.default_rng(d)
    lam0, mu0 = 1.3, 0.6
    xi = O.wavevectors(shape)
    u_hat = O.fft_r(rng.normal(size=(d,) + shape), shape)
    u_hat[:, O.zero_set(shape)] = 0.0
    E = rng.normal(size=(d, d)); E = 0.5 * (E + E.T)
    eps = O.ifft_r(O.sym_grad_hat(u_hat, xi), shape) + E.reshape((d, d) + (1,) * d)
    lhs = O.ifft_r(O.apply_U0(O.fft_r(O.stress(eps, lam0, mu0), shape), xi, lam0, mu0), shape)
    np.testing.assert_allclose(lhs, E.reshape((d, d) + (1,) * d) - eps, atol=1e-12)


@pytest.mark.parametrize("shape,m", [((16, 16), (3, -2)), ((8, 8, 8), (1, 2, -3))])
def test_homogeneous_plane_wave_closed_form(shape, m):
    """Homogeneous medium, single-mode force f = a cos(xi.x): exact
    u = [n n/((lam+2mu)|xi|^2) + (I - n n)/(mu |xi|^2)] a cos(xi.x); Algorithm 1
    stops after zero Green updates with eps = eps^b (P1)."""
    d = len(shape)
    lame = np.array([[1.1, 0.7]])
    phase = np.zeros(shape, dtype=np.uint8)
    pos = gen.grid_positions(shape)
    xi_vec = np.array([2 * np.pi * m[a] / shape[d - 1 - a] for a in range(d)])   # x first
    arg = sum(xi_vec[a] * pos[d - 1 - a] for a in range(d))
    a_vec = np.array([0.3, -1.0, 0.5][:d])
    f = np.stack([a_vec[c] * np.cos(arg) for c in range(d)])
    lam, mu = lame[0]
    n = xi_vec / np.linalg.norm(xi_vec)
    k2 = xi_vec @ xi_vec
    N = np.outer(n, n) / ((lam + 2 * mu) * k2) + (np.eye(d) - np.outer(n, n)) / (mu * k2)
    u_exact = np.stack([(N @ a_vec)[c] * np.cos(arg) for c in range(d)])
    res = O.solve_basic(phase, lame, f, tol=1e-12)
    assert res.iters == 0
    np.testing.assert_allclose(res.u, u_exact, atol=1e-13)


def test_scaled_reference_converges_to_closed_form():
    """L = alpha L0: the scheme converges geometrically to u = N0 f / alpha (P1)."""
    shape = (16, 16)
    lame = np.array([[2.0, 1.0]])
    phase = np.zeros(shape, dtype=np.uint8)
    f = rand_force(shape, 5)
    res = O.solve_basic(phase, lame, f, lam0=2.0 / 1.5, mu0=1.0 / 1.5, tol=1e-13)
    ref = O.solve_basic(phase, lame, f, tol=1e-13)          # L0 = L: exact in one step
    assert ref.iters == 0 and res.iters > 5
    np.testing.assert_allclose(res.u, ref.u, atol=1e-12 * np.abs(ref.u).max())
    # geometric rate |1 - alpha| / alpha-ish: successive residual ratios are constant
    h = np.array(res.history[1:8])
    ratios = h[1:] / h[:-1]
    np.testing.assert_allclose(ratios, ratios[0], rtol=1e-6)


# ---------------------------------------------------------------- dense direct solve (P7)

@pytest.mark.parametrize("shape", [(8, 8), (16, 16), (4, 4, 4), (6, 6, 6)])
def test_dense_direct_solve_equals_iterative(shape):
    """Brute-force dense solve of the same discretisation (Eq. 5.5) equals
    Algorithm 1 run to 1e-13, its displacement form and the displacement CG."""
    phase = rand_phase(shape, 1)
    f = rand_force(shape, 2)
    u, e, s = dense.dense_solve(phase, LAME10, f)
    for solver in (O.solve_basic, O.solve_displacement_update, O.solve_pcg_displacement):
        r = solver(phase, LAME10, f, tol=1e-13)
        assert r.status == O.STATUS_OK
        assert O.relative_strain_error(r.eps, e) < 1e-10
        assert np.abs(r.u - u).max() < 1e-10 * np.abs(u).max()
        assert np.abs(r.sig - s).max() < 1e-10 * np.abs(s).max()


def test_algorithm2_strain_cg_reaches_same_fixed_point():
    shape = (8, 8)
    phase = rand_phase(shape, 3)
    f = rand_force(shape, 4)
    u, e, s = dense.dense_solve(phase, LAME10, f)
    r = O.solve_cg_strain(phase, LAME10, f, tol=1e-13)
    assert O.relative_strain_error(r.eps, e) < 1e-9


def test_dense_matrix_is_symmetric_and_spectral_derivative_antisymmetric():
    A, D = dense.assemble(rand_phase((6, 4), 0), LAME10)
    np.testing.assert_allclose(A, A.T, atol=1e-12)
    for Dm in D:
        np.testing.assert_allclose(Dm, -Dm.T, atol=1e-13)


# ---------------------------------------------------------------- laminate, bounds (P3, P4)

def laminate_closed_form(lame, fractions, d):
    """Exact laminate (layers normal to x) in the Mandel basis: in-plane
    strains and normal tractions uniform; harmonic/arithmetic means of
    M = lam + 2 mu, mu and lam / M."""
    lam, mu = lame[:, 0], lame[:, 1]
    c = np.asarray(fractions)
    M = lam + 2 * mu
    av = lambda q: float(np.sum(c * q))
    h = av(1 / M)
    L = {}
    L["1111"] = 1 / h
    L["1122"] = av(lam / M) / h
    L["2222"] = av(lam / M) ** 2 / h - av(lam ** 2 / M) + av(M)
    L["2233"] = av(lam / M) ** 2 / h - av(lam ** 2 / M) + av(lam)
    mu12 = 1 / av(1 / mu)
    mu23 = av(mu)
    if d == 2:
        return np.array([[L["1111"], L["1122"], 0], [L["1122"], L["2222"], 0], [0, 0, 2 * mu12]])
    out = np.zeros((6, 6))
    out[0, 0] = L["1111"]
    out[0, 1] = out[1, 0] = out[0, 2] = out[2, 0] = L["1122"]
    out[1, 1] = out[2, 2] = L["2222"]
    out[1, 2] = out[2, 1] = L["2233"]
    out[3, 3] = 2 * mu23          # Mandel (23)
    out[4, 4] = 2 * mu12          # (13)
    out[5, 5] = 2 * mu12          # (12)
    return out


@pytest.mark.parametrize("shape", [(8, 16), (4, 4, 12)])
def test_laminate_effective_stiffness_closed_form(shape):
    """Classical mode on an even-width laminate reproduces the exact
    laminate stiffness (Eq. 6.3 with the closed form) (P3)."""
    d = len(shape)
    widths = [6, 10] if d == 2 else [4, 8]
    phase = gen.laminate(shape, widths)
    frac = [widths[0] / sum(widths), widths[1] / sum(widths)]
    L = O.effective_stiffness(phase, LAME10, tol=1e-12)
    np.testing.assert_allclose(L, laminate_closed_form(LAME10, frac, d), rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("shape", [(16, 16), (6, 6, 6)])
def test_voigt_reuss_bounds(shape):
    """L* is symmetric positive definite and lies between the Reuss and
    Voigt bounds (P4)."""
    d = len(shape)
    phase = rand_phase(shape, 7, 0.4)
    L = O.effective_stiffness(phase, LAME10, tol=1e-11)
    np.testing.assert_allclose(L, L.T, atol=1e-8 * np.abs(L).max())
    Ls = [O.stiffness_mandel(l, m, d) for l, m in LAME10]
    c = np.array([(phase == 0).mean(), (phase == 1).mean()])
    voigt = c[0] * Ls[0] + c[1] * Ls[1]
    reuss = np.linalg.inv(c[0] * np.linalg.inv(Ls[0]) + c[1] * np.linalg.inv(Ls[1]))
    assert np.linalg.eigvalsh(0.5 * (L + L.T)).min() > 0
    assert np.linalg.eigvalsh(voigt - 0.5 * (L + L.T)).min() > 1e-6
    assert np.linalg.eigvalsh(0.5 * (L + L.T) - reuss).min() > 1e-6


# ---------------------------------------------------------------- invariants (P5, P6, P8)

def test_invariants_at_return():
    """At return: Delta <= tol; eps = sym grad u (dense derivative matrices);
    sigma = L eps; div sigma = -P f to tol; Clapeyron and Betti (P5)."""
    shape = (16, 16)
    phase = rand_phase(shape, 11)
    f1, f2 = rand_force(shape, 12), rand_force(shape, 13)
    tol = 1e-10
    r1 = O.solve_basic(phase, LAME10, f1, tol=tol)
    r2 = O.solve_basic(phase, LAME10, f2, tol=tol)
    assert r1.residual <= tol
    D = [dense.axis_operator(shape, 1 - a, dense.derivative_matrix_1d(shape[1 - a])) for a in range(2)]
    npts = 256
    uc = r1.u.reshape(2, npts)
    for i in range(2):
        for j in range(2):
            e = 0.5 * (D[i] @ uc[j] + D[j] @ uc[i])
            np.testing.assert_allclose(e, r1.eps[i, j].ravel(), atol=1e-12)
    lam, mu = O.field_moduli(phase, LAME10)
    np.testing.assert_allclose(r1.sig, O.stress(r1.eps, lam, mu), atol=1e-14)
    P = dense.zero_mode_projector(shape)
    pf1 = np.stack([(P @ f1[c].ravel()).reshape(shape) for c in range(2)])
    pf2 = np.stack([(P @ f2[c].ravel()).reshape(shape) for c in range(2)])
    div = np.stack([sum(D[j] @ r1.sig[i, j].ravel() for j in range(2)) for i in range(2)]).reshape(pf1.shape)
    assert np.linalg.norm(div + pf1) <= 10 * tol * np.linalg.norm(pf1)
    # the stopping residual equals the real-space L2 ratio (Parseval weights)
    real_ratio = np.linalg.norm(div + pf1) / np.linalg.norm(pf1)
    assert abs(real_ratio - r1.residual) <= 1e-6 * r1.residual
    # removed mean is the voxel mean of the force
    np.testing.assert_allclose(r1.removed_mean, f1.reshape(2, -1).mean(axis=1), atol=1e-15)
    energy = np.sum(r1.sig * r1.eps)
    work = np.sum(pf1 * r1.u)
    assert abs(energy - work) <= 1e-8 * abs(work)
    assert abs(np.sum(f1 * r2.u) - np.sum(f2 * r1.u)) <= 1e-8 * abs(np.sum(f1 * r2.u))


def test_reference_medium_independence_and_linearity():
    """Two admissible reference media give the same solution; the solution is
    linear in the force (P6)."""
    shape = (16, 16)
    phase = rand_phase(shape, 21)
    f1, f2 = rand_force(shape, 22), rand_force(shape, 23)
    tol = 1e-11
    a = O.solve_basic(phase, LAME10, f1, tol=tol)
    lam0, mu0 = O.reference_medium(LAME10)
    b = O.solve_basic(phase, LAME10, f1, lam0=1.2 * lam0, mu0=1.2 * mu0, tol=tol)
    assert O.relative_strain_error(b.eps, a.eps) < 1e-8
    c = O.solve_basic(phase, LAME10, 2.0 * f1 - 3.0 * f2, tol=tol)
    d = O.solve_basic(phase, LAME10, f2, tol=tol)
    assert O.relative_strain_error(c.eps, 2.0 * a.eps - 3.0 * d.eps) < 1e-8


@pytest.mark.parametrize("shape,s", [((16, 12), (3, -5)), ((6, 8, 4), (1, 3, 2))])
def test_shift_covariance(shape, s):
    """Rolling phase map and force by the same integer shift rolls the
    solution (periodicity, Eqs. 2.7 and 2.21) (P8)."""
    d = len(shape)
    phase = rand_phase(shape, 31)
    f = rand_force(shape, 32)
    ax = tuple(range(d))
    a = O.solve_basic(phase, LAME10, f, tol=1e-11)
    b = O.solve_basic(np.roll(phase, s, ax), LAME10, np.roll(f, s, tuple(a_ + 1 for a_ in ax)), tol=1e-11)
    np.testing.assert_allclose(b.u, np.roll(a.u, s, tuple(a_ + 1 for a_ in ax)), atol=1e-10)
    assert b.iters == a.iters


def test_3d_invariant_along_z_equals_plane_strain():
    """A 3D problem with no dependence on z and no z force equals the 2D
    plane-strain problem (u_z = 0, eps_33 = 0, sigma_33 = lam tr eps)."""
    phase2 = rand_phase((8, 12), 41)
    f2 = rand_force((8, 12), 42)
    r2 = O.solve_basic(phase2, LAME10, f2, tol=1e-12)
    phase3 = np.broadcast_to(phase2, (4, 8, 12)).copy()
    f3 = np.zeros((3, 4, 8, 12))
    f3[:2] = f2[:, None]
    r3 = O.solve_basic(phase3, LAME10, f3, tol=1e-12)
    np.testing.assert_allclose(r3.u[:2], np.broadcast_to(r2.u[:, None], (2, 4, 8, 12)), atol=1e-11)
    assert np.abs(r3.u[2]).max() < 1e-12
    np.testing.assert_allclose(r3.eps[:2, :2], np.broadcast_to(r2.eps[:, :, None], (2, 2, 4, 8, 12)), atol=1e-11)


# ---------------------------------------------------------------- translated averaging (P9)

def _avg_setup():
    shape = (16, 16)
    phase = gen.tile_cell(gen.inclusion_per_cell((8, 8), 8, 0.25)[0], shape)
    return shape, phase


def test_average_homogeneous_equals_single_solve():
    shape = (16, 16)
    phase = np.zeros(shape, dtype=np.uint8)
    lame = np.array([[1.0, 0.5], [1.0, 0.5]])
    f = gen.bump_force(shape, (7.3, 8.1), 5.0, [0.6, 0.8])
    avg, _ = O.translate_average(phase, lame, f, gen.sample_shifts(8, 2, 6, 0), tol=1e-11)
    single = O.solve_basic(phase, lame, f, tol=1e-11)
    np.testing.assert_allclose(avg[0:2], single.u, atol=1e-14)
    np.testing.assert_allclose(avg[4:7], O.to_voigt(single.eps), atol=1e-14)
    assert np.abs(avg[-1]).max() == 0.0


@pytest.mark.slow
def test_average_full_set_invariants():
    """Full shift set over one cell: occupancy = cell volume fraction
    everywhere; translation equivariance of the averaged operator;
    reciprocity; and the force-shift implementation equals the literal
    microstructure shift (P9)."""
    shape, phase = _avg_setup()
    vf = phase.mean()
    shifts = gen.all_shifts(8, 2)
    f1 = gen.bump_force(shape, (7.0, 6.0), 4.5, [1.0, 0.0])
    f2 = gen.bump_force(shape, (3.0, 10.0), 4.0, [0.0, 1.0])
    tol = 1e-11
    a1, _ = O.translate_average(phase, LAME10, f1, shifts, tol=tol)
    a2, _ = O.translate_average(phase, LAME10, f2, shifts, tol=tol)
    np.testing.assert_allclose(a1[-1], vf, atol=1e-14)
    s = (3, 5)
    a1s, _ = O.translate_average(phase, LAME10, np.roll(f1, s, (1, 2)), shifts, tol=tol)
    np.testing.assert_allclose(a1s, np.roll(a1, s, (1, 2)), atol=1e-9 * np.abs(a1[:2]).max())
    lhs = np.sum(f2 * a1[0:2])
    rhs = np.sum(f1 * a2[0:2])
    assert abs(lhs - rhs) <= 1e-8 * abs(lhs)
    # force-shift rule: solve (phase, f(. + chi)) and read the output at x - chi
    for chi in shifts[::13]:
        chi = tuple(int(c) for c in chi)
        lit = O.solve_basic(np.roll(phase, chi, (0, 1)), LAME10, f1, tol=tol)
        neg = tuple(-c for c in chi)
        alt = O.solve_basic(phase, LAME10, np.roll(f1, neg, (1, 2)), tol=tol)
        np.testing.assert_allclose(np.roll(alt.u, chi, (1, 2)), lit.u, atol=1e-13)


def test_average_shift_direction_and_phase_hooke_invariants():
    """Eq. 3.3 moves the microstructure by +chi: phase_chi(x) = phase(x - chi),
    checked with explicit index arithmetic on the occupancy; on each phase
    Hooke's law holds for the restricted averages:
    <sigma>^(1) = L_incl <eps>^(1) and <sigma> - <sigma>^(1) = L_mat (<eps> - <eps>^(1));
    with one shift the restricted displacement is u V (P9)."""
    shape, phase = (16, 16), gen.tile_cell(gen.inclusion_per_cell((8, 8), 8, 0.25)[0], (16, 16))
    phase = phase.copy()
    phase[0, 1] = 1            # break the cell symmetry so direction matters
    f = gen.bump_force(shape, (6.2, 9.4), 5.0, [0.8, -0.6])
    shifts = np.array([[1, 3], [5, 2], [7, 6]], dtype=np.int32)
    avg, _ = O.translate_average(phase, LAME10, f, shifts, tol=1e-11)
    occ = np.zeros(shape)
    for (cy, cx) in shifts:
        for y in range(16):
            for x in range(16):
                occ[y, x] += phase[(y - cy) % 16, (x - cx) % 16] == 1
    np.testing.assert_allclose(avg[-1], occ / len(shifts), atol=1e-15)
    d, s = 2, 3
    e0, e1 = avg[2 * d:2 * d + s], avg[2 * d + s:2 * d + 2 * s]
    s0, s1 = avg[2 * d + 2 * s:2 * d + 3 * s], avg[2 * d + 3 * s:2 * d + 4 * s]

    def hooke(ev, lam, mu):
        t = O.from_voigt(ev, d)
        return O.to_voigt(O.stress(t, lam, mu))

    np.testing.assert_allclose(s1, hooke(e1, *LAME10[1]), atol=1e-13)
    np.testing.assert_allclose(s0 - s1, hooke(e0 - e1, *LAME10[0]), atol=1e-13)
    one, _ = O.translate_average(phase, LAME10, f, shifts[:1], tol=1e-11)
    ref = O.solve_basic(np.roll(phase, (1, 3), (0, 1)), LAME10, f, tol=1e-11)
    ind = np.roll(phase, (1, 3), (0, 1)) == 1
    np.testing.assert_allclose(one[2:4], ref.u * ind, atol=1e-15)


def test_warm_start_from_the_solution_and_from_a_shifted_start():
    # started at its own converged displacement the iteration stops at once
    # with the same fields; from any other start it reaches the same
    # solution (the fixed point does not depend on the start)
    shape = (16, 12)
    phase = (np.random.default_rng(71).random(shape) < 0.4).astype(np.uint8)
    f = np.random.default_rng(72).normal(size=(2,) + shape)
    cold = O.solve_displacement_update(phase, LAME10, f, tol=1e-12)
    warm = O.solve_displacement_update(phase, LAME10, f, tol=1e-10, u_init=cold.u)
    assert warm.iters == 0
    np.testing.assert_allclose(warm.eps, cold.eps, rtol=0, atol=1e-11 * np.abs(cold.eps).max())
    rnd = O.solve_displacement_update(phase, LAME10, f, tol=1e-12,
                                      u_init=np.random.default_rng(73).normal(size=(2,) + shape) + 5.0)
    np.testing.assert_allclose(rnd.eps, cold.eps, rtol=0, atol=1e-9 * np.abs(cold.eps).max())
    # the mean of the start is dropped: a uniform shift of the start changes nothing
    a = O.solve_displacement_update(phase, LAME10, f, tol=1e-10, max_iter=3, u_init=cold.u * 0.5)
    b = O.solve_displacement_update(phase, LAME10, f, tol=1e-10, max_iter=3, u_init=cold.u * 0.5 + 3.0)
    np.testing.assert_allclose(a.eps, b.eps, rtol=0, atol=1e-13 * np.abs(a.eps).max())
    np.testing.assert_allclose(a.u, b.u, rtol=0, atol=1e-13 * np.abs(a.u).max())
