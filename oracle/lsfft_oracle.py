"""Plain float64 NumPy oracle of the BFCS modified Lippmann-Schwinger method.

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

Every function follows a passage of Buryachenko, "New RVE concept and FFT
methods in micromechanics of composites subjected to body force with compact
support" (arXiv 2601.00822); the passage is named in its docstring.  Readings
taken where the paper is silent or garbled:

* Frequencies: node ``k`` at ``x = k h`` with ``h = 1`` (Eq. 4.1); the
  wavevector along an axis of ``N`` nodes is ``xi = 2 pi kt / N`` with signed
  ``kt`` in ``[-N/2, N/2)``; on the Nyquist index ``kt = -N/2`` the wavevector
  component is set to zero, so every spectral operator maps real fields to
  real fields.  ``Z`` is the set of modes with ``xi = 0`` (the mean and the
  pure-Nyquist corners); the force is projected off ``Z`` and its removed mean
  is reported (Eq. 2.5 asks for a self-equilibrated force; a one-signed bump is
  not).
* Transforms follow Eqs. 4.3-4.5: forward unnormalised with ``exp(-i...)``,
  inverse with ``1/|N|``; the real-to-half-spectrum layout keeps x last.
* The strain Green operator is ``U0 = -Gamma0`` (Eqs. 2.16-2.18 with the
  garbled index ``h`` read as ``l``); written through the inverse acoustic
  tensor ``N0 = K0^{-1}``, ``K0 = mu0 |xi|^2 I + (lam0 + mu0) xi xi^T``, the
  same operator is ``U0 tau = sym(i xi (x) N0 (i xi . tau))``.
* Stopping rule under body force (Eq. 5.11 divides by the mean stress, which
  vanishes here): ``Delta = ||i xi . sigma^ + P f^|| / ||P f^||`` with
  Parseval weights on the half spectrum.  The classical mode keeps Eq. 5.11
  as printed.
* The returned iterate is the first ``j`` with ``Delta_j <= tol``; the
  iteration count is the number of Green updates applied.
* Tensors are full ``d x d`` here; results are also given in Voigt order
  (11,22,33,23,13,12) in 3D and (11,22,12) in 2D, tensor (not engineering)
  shear.  2D is plane strain.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

STATUS_OK = 0
STATUS_NOCONV = -4

VOIGT = {2: [(0, 0), (1, 1), (0, 1)],
         3: [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]}


# --------------------------------------------------------------------------
# Material data (Sec. 2, the isotropic stiffness after Eq. 2.3)
# --------------------------------------------------------------------------

def lame_from_young(table) -> np.ndarray:
    """``[nphase][2]`` of ``(E, nu)`` to ``(lambda, mu)`` (3D Lame constants).

    Plane strain uses the same pair; the isotropic stiffness is
    ``L = (d k, 2 mu)`` with ``lambda = k - 2 mu / d`` (Sec. 2).
    """
    t = np.asarray(table, dtype=np.float64)
    e, nu = t[:, 0], t[:, 1]
    lam = e * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = e / (2.0 * (1.0 + nu))
    return np.stack([lam, mu], axis=1)


def reference_medium(lame) -> tuple[float, float]:
    """Reference medium ``L0`` (a datum of Algorithm 1): mean of the extreme
    Lame constants over the phases."""
    lame = np.asarray(lame, dtype=np.float64)
    lam0 = 0.5 * (lame[:, 0].min() + lame[:, 0].max())
    mu0 = 0.5 * (lame[:, 1].min() + lame[:, 1].max())
    return float(lam0), float(mu0)


# --------------------------------------------------------------------------
# Discrete Fourier transform (Sec. 4, Eqs. 4.1-4.10)
# --------------------------------------------------------------------------

def _spatial_axes(shape):
    return tuple(range(1, len(shape) + 1))


def fft_r(a, shape):
    """Forward DFT (Eq. 4.3) of real fields ``[..comp..][grid]`` onto the half spectrum."""
    lead = a.ndim - len(shape)
    return np.fft.rfftn(a, axes=tuple(range(lead, a.ndim)))


def ifft_r(a, shape):
    """Inverse DFT (Eq. 4.4) from the half spectrum back to real fields."""
    lead = a.ndim - len(shape)
    return np.fft.irfftn(a, s=shape, axes=tuple(range(lead, a.ndim)))


def wavevectors(shape):
    """Wavevector components ``xi_alpha`` (alpha = 0 is x, the last array axis),
    each broadcastable to the half-spectrum shape; Nyquist components are 0."""
    d = len(shape)
    spec = list(shape[:-1]) + [shape[-1] // 2 + 1]
    xi = []
    for alpha in range(d):
        ax = d - 1 - alpha          # array axis of spatial direction alpha
        n = shape[ax]
        if ax == d - 1:
            kt = np.arange(n // 2 + 1, dtype=np.float64)
        else:
            kt = np.fft.fftfreq(n) * n
        kt = np.where(np.abs(kt) == n // 2, 0.0, kt)
        v = 2.0 * np.pi * kt / n
        s = [1] * d
        s[ax] = spec[ax]
        xi.append(v.reshape(s))
    return xi


def hermitian_weights(shape):
    """Parseval weights of the half spectrum: 1 on the ``kx = 0`` and
    ``kx = Nx/2`` planes, 2 elsewhere."""
    nxh = shape[-1] // 2 + 1
    w = np.full(nxh, 2.0)
    w[0] = 1.0
    w[-1] = 1.0
    s = [1] * len(shape)
    s[-1] = nxh
    return w.reshape(s)


def zero_set(shape):
    """Mask of half-spectrum modes with ``xi = 0``."""
    xi = wavevectors(shape)
    m = np.ones(np.broadcast_shapes(*[x.shape for x in xi]), dtype=bool)
    for x in xi:
        m = m & (x == 0.0)
    return m


# --------------------------------------------------------------------------
# Green operators (Sec. 2, Eqs. 2.6-2.9, 2.14, 2.16-2.18)
# --------------------------------------------------------------------------

def apply_N0(v_hat, xi, lam0, mu0):
    """Inverse acoustic tensor of the reference medium applied to a vector
    spectrum: ``N0 v = (v - c0 xi (xi . v) / |xi|^2) / (mu0 |xi|^2)`` with
    ``c0 = (lam0 + mu0) / (lam0 + 2 mu0)``; zero where ``xi = 0``.
    ``N0`` is the Fourier symbol of the periodic displacement Green operator
    ``G0`` of Eq. 2.9 (``-L0 grad grad`` inverted)."""
    d = len(xi)
    xi2 = sum(x * x for x in xi)
    safe = np.where(xi2 == 0.0, 1.0, xi2)
    c0 = (lam0 + mu0) / (lam0 + 2.0 * mu0)
    xv = sum(xi[a] * v_hat[a] for a in range(d))
    out = np.empty(np.broadcast_shapes(v_hat.shape, (d,) + xi2.shape), dtype=np.complex128)
    for a in range(d):
        out[a] = (v_hat[a] - c0 * xi[a] * xv / safe) / (mu0 * safe)
        out[a] = np.where(xi2 == 0.0, 0.0, out[a])
    return out


def sym_grad_hat(u_hat, xi):
    """Spectral symmetric gradient ``eps^_ij = (i/2)(xi_i u^_j + xi_j u^_i)``
    (Eq. 2.3 with the derivative rule Eq. 4.8)."""
    d = len(xi)
    e = np.empty((d, d) + u_hat.shape[1:], dtype=np.complex128)
    for i in range(d):
        for j in range(d):
            e[i, j] = 0.5j * (xi[i] * u_hat[j] + xi[j] * u_hat[i])
    return e


def div_hat(s_hat, xi):
    """Spectral divergence of a tensor field ``(i xi_j s^_ij)_i`` (Eq. 2.1)."""
    d = len(xi)
    return np.stack([sum(1j * xi[j] * s_hat[i, j] for j in range(d)) for i in range(d)])


def apply_U0(tau_hat, xi, lam0, mu0):
    """Strain Green operator of Eq. 2.14 in Fourier space:
    ``U0 tau^ = sym(i xi (x) N0 (i xi . tau^))`` = ``-Gamma0 tau^``; zero on ``Z``."""
    return sym_grad_hat(apply_N0(div_hat(tau_hat, xi), xi, lam0, mu0), xi)


# --------------------------------------------------------------------------
# Local constitutive law (Eq. 2.2) and Voigt packing
# --------------------------------------------------------------------------

def stress(eps, lam, mu):
    """``sigma = lam tr(eps) I + 2 mu eps`` for full ``d x d`` tensor fields."""
    d = eps.shape[0]
    tr = sum(eps[i, i] for i in range(d))
    s = 2.0 * mu * eps
    for i in range(d):
        s[i, i] = s[i, i] + lam * tr
    return s


def to_voigt(t):
    d = t.shape[0]
    return np.stack([t[i, j] for (i, j) in VOIGT[d]])


def from_voigt(v, d):
    t = np.empty((d, d) + v.shape[1:], dtype=v.dtype)
    for c, (i, j) in enumerate(VOIGT[d]):
        t[i, j] = v[c]
        t[j, i] = v[c]
    return t


def field_moduli(phase, lame):
    lame = np.asarray(lame, dtype=np.float64)
    return lame[phase, 0], lame[phase, 1]


# --------------------------------------------------------------------------
# Results
# --------------------------------------------------------------------------

@dataclass
class Result:
    eps: np.ndarray            # [d][d][grid]
    sig: np.ndarray            # [d][d][grid]
    u: np.ndarray              # [d][grid]
    iters: int
    residual: float
    history: list = field(default_factory=list)
    removed_mean: np.ndarray = None
    status: int = STATUS_OK

    @property
    def eps_voigt(self):
        return to_voigt(self.eps)

    @property
    def sig_voigt(self):
        return to_voigt(self.sig)


def _norm_w(v_hat, w):
    return float(np.sqrt(np.sum(w * np.abs(v_hat) ** 2)))


def _prepare(phase, lame, f, lam0, mu0):
    phase = np.asarray(phase)
    shape = phase.shape
    if lam0 is None or mu0 is None:
        lam0, mu0 = reference_medium(lame)
    lam, mu = field_moduli(phase, lame)
    xi = wavevectors(shape)
    w = hermitian_weights(shape)
    zmask = zero_set(shape)
    f_hat = fft_r(np.asarray(f, dtype=np.float64), shape)
    n_tot = float(np.prod(shape))
    origin = (slice(None),) + (0,) * len(shape)
    removed = f_hat[origin].real / n_tot
    f_hat[:, zmask] = 0.0
    return shape, lam0, mu0, lam, mu, xi, w, f_hat, removed


# --------------------------------------------------------------------------
# Algorithm 1: modified basic scheme (Sec. 5, Eqs. 5.7-5.11)
# --------------------------------------------------------------------------

def free_term(f_hat, xi, shape, lam0, mu0):
    """Reference-medium response to the force (Eqs. 2.8-2.9):
    ``u^b = N0 f^``, ``eps^b = sym grad u^b`` (Eq. 2.14's free term)."""
    ub_hat = apply_N0(f_hat, xi, lam0, mu0)
    eb_hat = sym_grad_hat(ub_hat, xi)
    return ub_hat, eb_hat, ifft_r(ub_hat, shape), ifft_r(eb_hat, shape)


def solve_basic(phase, lame, f, lam0=None, mu0=None, tol=1e-8, max_iter=10000):
    """Algorithm 1 (modified basic scheme) as printed, step by step:

    start from ``eps^0 = eps^b`` (and ``u^0 = u^b``); while the equilibrium
    residual exceeds ``tol``: polarization ``tau = L1 eps`` (Eq. 5.7), its DFT
    (Eq. 5.8), ``eps^ = U0 tau^`` off ``Z`` (Eq. 5.9), and
    ``eps = F^{-1} eps^ + eps^b`` (Eq. 5.10).  The displacement is carried
    along as ``u = F^{-1}(N0 (i xi . tau^)) + u^b`` (Eq. 2.10).
    """
    shape, lam0, mu0, lam, mu, xi, w, f_hat, removed = _prepare(phase, lame, f, lam0, mu0)
    d = len(shape)
    fnorm = _norm_w(f_hat, w)
    ub_hat, eb_hat, ub, eb = free_term(f_hat, xi, shape, lam0, mu0)
    eps, u = eb.copy(), ub.copy()
    if fnorm == 0.0:
        z = np.zeros_like(eps)
        return Result(z, z.copy(), np.zeros_like(u), 0, 0.0, [0.0], removed, STATUS_OK)
    j = 0
    hist = []
    while True:
        sig = stress(eps, lam, mu)
        r_hat = div_hat(fft_r(sig, shape), xi) + f_hat
        delta = _norm_w(r_hat, w) / fnorm
        hist.append(delta)
        if delta <= tol or j >= max_iter:
            break
        tau = stress(eps, lam - lam0, mu - mu0)                 # Eq. 5.7
        tau_hat = fft_r(tau, shape)                              # Eq. 5.8
        w_hat = apply_N0(div_hat(tau_hat, xi), xi, lam0, mu0)
        e_hat = sym_grad_hat(w_hat, xi)                          # Eq. 5.9 (U0 tau^)
        eps = ifft_r(e_hat, shape) + eb                          # Eq. 5.10
        u = ifft_r(w_hat, shape) + ub
        j += 1
    status = STATUS_OK if delta <= tol else STATUS_NOCONV
    return Result(eps, stress(eps, lam, mu), u, j, delta, hist, removed, status)


def solve_displacement_update(phase, lame, f, lam0=None, mu0=None, tol=1e-8, max_iter=10000, u_init=None):
    """The same iteration written on the displacement spectrum:
    ``u^{j+1} = u^j + N0 (i xi . sigma^j + f^)``.  This is Algorithm 1 after
    the identity of Eq. 2.27 (``U0 (L0 eps) = -eps`` for compatible mean-free
    ``eps``), i.e. the body-force analogue of the recurrence Eq. 2.28.  It
    pins that equivalence, and with ``u_init`` (a real ``[d][grid]`` field)
    it starts from that displacement instead of the free term: its spectrum,
    zeroed where xi = 0 like the force (the mean displacement is free)."""
    shape, lam0, mu0, lam, mu, xi, w, f_hat, removed = _prepare(phase, lame, f, lam0, mu0)
    fnorm = _norm_w(f_hat, w)
    if u_init is None:
        u_hat = apply_N0(f_hat, xi, lam0, mu0)
    else:
        u_hat = fft_r(np.asarray(u_init, dtype=np.float64), shape)
        u_hat[:, zero_set(shape)] = 0.0
    j = 0
    hist = []
    while True:
        eps = ifft_r(sym_grad_hat(u_hat, xi), shape)
        sig = stress(eps, lam, mu)
        r_hat = div_hat(fft_r(sig, shape), xi) + f_hat
        delta = _norm_w(r_hat, w) / fnorm if fnorm > 0 else 0.0
        hist.append(delta)
        if delta <= tol or j >= max_iter:
            break
        u_hat = u_hat + apply_N0(r_hat, xi, lam0, mu0)
        j += 1
    status = STATUS_OK if delta <= tol else STATUS_NOCONV
    return Result(eps, sig, ifft_r(u_hat, shape), j, delta, hist, removed, status)


# --------------------------------------------------------------------------
# Algorithm 2 (Krylov form, Eqs. 5.12-5.13) and the displacement CG
# (Eqs. 5.14-5.22)
# --------------------------------------------------------------------------

def solve_cg_strain(phase, lame, f, lam0=None, mu0=None, tol=1e-8, max_iter=2000):
    """Algorithm 2 as printed: conjugate gradients on
    ``A(eps) = eps - F^{-1}{U0 : F[L1 : eps]}`` with right-hand side
    ``eps^b`` and ``eps = 0`` to start, using the plain Euclidean inner
    product ``sum_x eps : eps``.  Stops when ``||b - A eps|| <= tol ||eps^b||``.
    Returned ``residual`` is the equilibrium residual of the result."""
    shape, lam0, mu0, lam, mu, xi, w, f_hat, removed = _prepare(phase, lame, f, lam0, mu0)
    fnorm = _norm_w(f_hat, w)
    _, _, ub, eb = free_term(f_hat, xi, shape, lam0, mu0)

    def op(e):
        return e - ifft_r(apply_U0(fft_r(stress(e, lam - lam0, mu - mu0), shape), xi, lam0, mu0), shape)

    def dot(a, b):
        return float(np.sum(a * b))

    eps = np.zeros_like(eb)
    r = eb - op(eps)
    p = r.copy()
    rr = dot(r, r)
    bnorm = np.sqrt(dot(eb, eb))
    j = 0
    while np.sqrt(rr) > tol * bnorm and j < max_iter:
        ap = op(p)
        alpha = rr / dot(p, ap)
        eps = eps + alpha * p
        r = r - alpha * ap
        rr_new = dot(r, r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        j += 1
    sig = stress(eps, lam, mu)
    r_hat = div_hat(fft_r(sig, shape), xi) + f_hat
    delta = _norm_w(r_hat, w) / fnorm if fnorm > 0 else 0.0
    # displacement of the strain iterate: eps - eps^b is compatible, recover u1
    e1_hat = fft_r(eps - eb, shape)
    u1_hat = _displacement_from_strain_hat(e1_hat, xi)
    u = ifft_r(u1_hat, shape) + ub
    status = STATUS_OK if np.sqrt(rr) <= tol * bnorm else STATUS_NOCONV
    return Result(eps, sig, u, j, delta, [], removed, status)


def _displacement_from_strain_hat(e_hat, xi):
    """Least-squares ``u^`` with ``sym(i xi (x) u^) = e^`` (exact for
    compatible ``e``): ``u^ = -i (2 e^ xi - (xi . e^ xi) xi / |xi|^2) / |xi|^2``."""
    d = len(xi)
    xi2 = sum(x * x for x in xi)
    safe = np.where(xi2 == 0.0, 1.0, xi2)
    ex = np.stack([sum(e_hat[i, j] * xi[j] for j in range(d)) for i in range(d)])
    xex = sum(xi[i] * ex[i] for i in range(d))
    u = np.stack([-1j * (2.0 * ex[i] - xex * xi[i] / safe) / safe for i in range(d)])
    return np.where(xi2 == 0.0, 0.0, u)


def solve_pcg_displacement(phase, lame, f, lam0=None, mu0=None, tol=1e-8, max_iter=5000):
    """Conjugate gradients on the displacement form of the equilibrium
    equation (Eqs. 5.14-5.17; right-hand side read as ``-div(L1 eps^b)``, the
    printed ``-div(L eps^b)`` drops the force): unknown ``u = u^b + u1`` with
    ``u1 = 0`` to start, operator ``A u = -div(L sym grad u)`` (symmetric
    positive semi-definite, null on ``Z``), residual ``r = P f + div(L sym
    grad u)``, preconditioner ``N0`` (the reference-medium inverse), and the
    CG updates of Eqs. 5.18-5.22 with the preconditioned inner products
    ``r.z`` (Parseval-weighted half-spectrum sums).  Stops when
    ``||r|| / ||P f|| <= tol``."""
    shape, lam0, mu0, lam, mu, xi, w, f_hat, removed = _prepare(phase, lame, f, lam0, mu0)
    fnorm = _norm_w(f_hat, w)

    def a_op(v_hat):
        e = ifft_r(sym_grad_hat(v_hat, xi), shape)
        return -div_hat(fft_r(stress(e, lam, mu), shape), xi)

    def dot(a, b):
        return float(np.sum(w * (np.conj(a) * b).real))

    u_hat = apply_N0(f_hat, xi, lam0, mu0)
    r = f_hat - a_op(u_hat)
    z = apply_N0(r, xi, lam0, mu0)
    p = z.copy()
    rz = dot(r, z)
    j = 0
    hist = []
    while True:
        delta = np.sqrt(dot(r, r)) / fnorm if fnorm > 0 else 0.0
        hist.append(delta)
        if delta <= tol or j >= max_iter:
            break
        q = a_op(p)
        alpha = rz / dot(p, q)                                   # Eq. 5.18
        u_hat = u_hat + alpha * p                                # Eq. 5.19
        r = r - alpha * q                                        # Eq. 5.20
        z = apply_N0(r, xi, lam0, mu0)
        rz_new = dot(r, z)
        beta = rz_new / rz                                       # Eq. 5.21
        p = z + beta * p                                         # Eq. 5.22
        rz = rz_new
        j += 1
    eps = ifft_r(sym_grad_hat(u_hat, xi), shape)
    status = STATUS_OK if delta <= tol else STATUS_NOCONV
    return Result(eps, stress(eps, lam, mu), ifft_r(u_hat, shape), j, delta, hist, removed, status)


def solve_cg_alg3(phase, lame, f, lam0=None, mu0=None, tol=1e-8, max_iter=20000, start="printed"):
    """Algorithm 3 (Sec. 5, Eqs. 5.17-5.22): plain conjugate gradients, no
    preconditioner, on the displacement-fluctuation system ``A(u1) = b^A``
    of Eqs. 5.14-5.17, with ``A(v) = -div(L sym grad v)`` and
    ``b^A = div(L1 eps^b)`` (the printed right-hand side of Eq. 5.14 drops
    the force; with ``u = u^b + u1`` the residual ``b^A - A(u1)`` equals
    ``P f + div(L sym grad u)``).  The start is ``u1 = b^A`` as printed
    (``start="printed"``) or ``u1 = 0`` (``start="zero"``, the reading used
    where the printed start mixes a force with a displacement); then
    ``r = b^A - A(u1)``, ``p = r``, and per iteration
    ``alpha = r.r / p.A(p)`` (Eq. 5.18, ``A`` symmetric), ``u1 += alpha p``
    (5.19), ``r -= alpha A(p)`` (5.20), ``beta = r'.r' / r.r`` (5.21),
    ``p = r' + beta p`` (5.22).  Inner products are Parseval-weighted
    half-spectrum sums.  Stops when ``||r|| / ||P f|| <= tol``; the strain is
    ``sym grad(u^b + u1)`` (the printed ``u1 + eps^b``)."""
    shape, lam0, mu0, lam, mu, xi, w, f_hat, removed = _prepare(phase, lame, f, lam0, mu0)
    fnorm = _norm_w(f_hat, w)

    def a_op(v_hat):
        e = ifft_r(sym_grad_hat(v_hat, xi), shape)
        return -div_hat(fft_r(stress(e, lam, mu), shape), xi)

    def dot(a, b):
        return float(np.sum(w * (np.conj(a) * b).real))

    ub_hat = apply_N0(f_hat, xi, lam0, mu0)
    b_a = f_hat - a_op(ub_hat)                                   # b^A = r(u^b)
    if start == "printed":
        u1 = b_a.copy()
    elif start == "zero":
        u1 = np.zeros_like(b_a)
    else:
        raise ValueError("start is 'printed' or 'zero'")
    r = b_a - a_op(u1)
    p = r.copy()
    rr = dot(r, r)
    j = 0
    hist = []
    while True:
        delta = np.sqrt(rr) / fnorm if fnorm > 0 else 0.0
        hist.append(delta)
        if delta <= tol or j >= max_iter:
            break
        q = a_op(p)
        alpha = rr / dot(p, q)                                   # Eq. 5.18
        u1 = u1 + alpha * p                                      # Eq. 5.19
        r = r - alpha * q                                        # Eq. 5.20
        rr_new = dot(r, r)
        beta = rr_new / rr                                       # Eq. 5.21
        p = r + beta * p                                         # Eq. 5.22
        rr = rr_new
        j += 1
    u_hat = ub_hat + u1
    eps = ifft_r(sym_grad_hat(u_hat, xi), shape)
    status = STATUS_OK if delta <= tol else STATUS_NOCONV
    return Result(eps, stress(eps, lam, mu), ifft_r(u_hat, shape), j, delta, hist, removed, status)


# --------------------------------------------------------------------------
# Anderson acceleration of the basic scheme (Sec. 5 names accelerated
# schemes for high contrast; the method is Anderson's, in the form of
# Walker & Ni, SIAM J. Numer. Anal. 49 (2011))
# --------------------------------------------------------------------------

def solve_anderson(phase, lame, f, lam0=None, mu0=None, tol=1e-8, max_iter=10000, m=5):
    """Anderson acceleration with memory ``m`` and mixing 1 of the basic
    scheme's fixed-point map in displacement form,
    ``g(u) = u + N0 (i xi . sigma^(u) + f^)`` (Algorithm 1 after Eq. 2.27).
    With ``F_k = g(u_k) - u_k`` and the differences ``dF_i = F_{i+1} - F_i``,
    ``dU_i = u_{i+1} - u_i`` of the last ``m_k = min(m, k)`` steps:
    ``gamma = argmin || F_k - sum_i gamma_i dF_i ||`` (Parseval-weighted
    least squares) and ``u_{k+1} = u_k + F_k - sum_i gamma_i (dU_i + dF_i)``.
    ``m = 0`` is the basic scheme.  Starts at ``u^b``; stops when the
    equilibrium residual ``||i xi . sigma^ + P f^|| / ||P f^|| <= tol``;
    iterations = updates applied."""
    shape, lam0, mu0, lam, mu, xi, w, f_hat, removed = _prepare(phase, lame, f, lam0, mu0)
    fnorm = _norm_w(f_hat, w)
    sw = np.sqrt(w)

    def realvec(v_hat):
        # half-spectrum field as a real vector whose dot products are the
        # Parseval-weighted ones
        return np.concatenate([(sw * v_hat.real).ravel(), (sw * v_hat.imag).ravel()])

    u_hat = apply_N0(f_hat, xi, lam0, mu0)
    dU, dF = [], []
    u_prev = F_prev = None
    j = 0
    hist = []
    while True:
        eps = ifft_r(sym_grad_hat(u_hat, xi), shape)
        sig = stress(eps, lam, mu)
        r_hat = div_hat(fft_r(sig, shape), xi) + f_hat
        delta = _norm_w(r_hat, w) / fnorm if fnorm > 0 else 0.0
        hist.append(delta)
        if delta <= tol or j >= max_iter:
            break
        F = apply_N0(r_hat, xi, lam0, mu0)
        if F_prev is not None and m > 0:
            dU.append(u_hat - u_prev)
            dF.append(F - F_prev)
            if len(dF) > m:
                dU.pop(0)
                dF.pop(0)
        u_prev, F_prev = u_hat, F
        if dF:
            A = np.stack([realvec(v) for v in dF], axis=1)
            gamma = np.linalg.lstsq(A, realvec(F), rcond=None)[0]
            u_hat = u_hat + F - sum(g * (a + b) for g, a, b in zip(gamma, dU, dF))
        else:
            u_hat = u_hat + F
        j += 1
    status = STATUS_OK if delta <= tol else STATUS_NOCONV
    return Result(eps, sig, ifft_r(u_hat, shape), j, delta, hist, removed, status)


# --------------------------------------------------------------------------
# Classical Lippmann-Schwinger mode (Eqs. 2.24-2.26, 5.1-5.2, 5.11, 6.1-6.3)
# --------------------------------------------------------------------------

def solve_classical(phase, lame, macro_strain, lam0=None, mu0=None, tol=1e-10, max_iter=20000):
    """Basic scheme for the classical problem with prescribed mean strain
    ``E`` and no body force: ``eps^0 = E``; ``eps^ = U0 (L1 eps)^`` off the
    origin and ``eps^(0) = |N| E`` (Eq. 5.2); stop on Eq. 5.11 as printed:
    ``sqrt(sum_xi |xi . sigma^|^2) / |sigma^(0)|``."""
    phase = np.asarray(phase)
    shape = phase.shape
    d = len(shape)
    if lam0 is None or mu0 is None:
        lam0, mu0 = reference_medium(lame)
    lam, mu = field_moduli(phase, lame)
    xi = wavevectors(shape)
    w = hermitian_weights(shape)
    E = np.asarray(macro_strain, dtype=np.float64)
    n_tot = float(np.prod(shape))
    eps = np.broadcast_to(E.reshape((d, d) + (1,) * d), (d, d) + shape).copy()
    origin = (slice(None), slice(None)) + (0,) * d
    j = 0
    while True:
        sig = stress(eps, lam, mu)
        s_hat = fft_r(sig, shape)
        xs = np.stack([sum(xi[jj] * s_hat[i, jj] for jj in range(d)) for i in range(d)])
        num = np.sqrt(np.sum(w * np.abs(xs) ** 2))
        den = np.sqrt(np.sum(np.abs(s_hat[origin]) ** 2))
        delta = num / den if den > 0 else 0.0
        if delta <= tol or j >= max_iter:
            break
        tau_hat = fft_r(stress(eps, lam - lam0, mu - mu0), shape)
        e_hat = apply_U0(tau_hat, xi, lam0, mu0)
        e_hat[origin] = E * n_tot
        eps = ifft_r(e_hat, shape)
        j += 1
    status = STATUS_OK if delta <= tol else STATUS_NOCONV
    return Result(eps, stress(eps, lam, mu), None, j, delta, [], None, status)


def mandel_basis(d):
    """Orthonormal symmetric-tensor basis in Voigt order (shear entries 1/sqrt 2)."""
    out = []
    for (i, j) in VOIGT[d]:
        b = np.zeros((d, d))
        if i == j:
            b[i, i] = 1.0
        else:
            b[i, j] = b[j, i] = 1.0 / np.sqrt(2.0)
        out.append(b)
    return out


def effective_stiffness(phase, lame, lam0=None, mu0=None, tol=1e-11):
    """``L*`` in the Mandel basis from ``<sigma> = L* <eps>`` (Eq. 6.3) with one
    classical solve per basis strain."""
    phase = np.asarray(phase)
    d = phase.ndim
    basis = mandel_basis(d)
    m = len(basis)
    L = np.zeros((m, m))
    for b, E in enumerate(basis):
        res = solve_classical(phase, lame, E, lam0, mu0, tol=tol)
        mean_sig = res.sig.reshape(d, d, -1).mean(axis=-1)
        for a, B in enumerate(basis):
            L[a, b] = float(np.sum(B * mean_sig))
    return L


def stiffness_mandel(lam, mu, d):
    """Isotropic stiffness as a Mandel matrix."""
    basis = mandel_basis(d)
    m = len(basis)
    L = np.zeros((m, m))
    for b, E in enumerate(basis):
        S = lam * np.trace(E) * np.eye(d) + 2.0 * mu * E
        for a, B in enumerate(basis):
            L[a, b] = float(np.sum(B * S))
    return L


# --------------------------------------------------------------------------
# Translated averaging (Sec. 3, Eqs. 3.3-3.7)
# --------------------------------------------------------------------------

def average_components(d):
    """Names of the averaged fields in output order (Eq. 3.7 plus occupancy)."""
    s = len(VOIGT[d])
    return (["u"] * d + ["u1"] * d + ["eps"] * s + ["eps1"] * s
            + ["sig"] * s + ["sig1"] * s + ["occ"])


def translate_average(phase, lame, f, shifts, incl_phase=1, lam0=None, mu0=None,
                      tol=1e-8, max_iter=10000, solver=None):
    """Translated (ensemble) averages over rigid shifts of the microstructure
    with the force fixed (Eqs. 3.3-3.6): for each ``chi`` the phase map is
    ``phase_chi(x) = phase(x - chi)`` (Eq. 3.3), the problem is solved, and
    ``u``, ``u V``, ``eps``, ``eps V``, ``sigma``, ``sigma V`` and ``V`` are
    summed, ``V`` the indicator of ``incl_phase``; the sums are divided by the
    number of shifts (Eqs. 3.5-3.6).  Returns ``[2d + 4s + 1][grid]`` and the
    per-shift results' iteration counts."""
    phase = np.asarray(phase)
    shape = phase.shape
    d = len(shape)
    if lam0 is None or mu0 is None:
        lam0, mu0 = reference_medium(lame)
    solver = solver or solve_basic
    s = len(VOIGT[d])
    acc = np.zeros((2 * d + 4 * s + 1,) + shape)
    iters = []
    for chi in np.asarray(shifts).reshape(-1, d):
        ph = np.roll(phase, shift=tuple(int(c) for c in chi), axis=tuple(range(d)))
        res = solver(ph, lame, f, lam0, mu0, tol=tol, max_iter=max_iter)
        ind = (ph == incl_phase).astype(np.float64)
        ev, sv = to_voigt(res.eps), to_voigt(res.sig)
        k = 0
        acc[k:k + d] += res.u; k += d
        acc[k:k + d] += res.u * ind; k += d
        acc[k:k + s] += ev; k += s
        acc[k:k + s] += ev * ind; k += s
        acc[k:k + s] += sv; k += s
        acc[k:k + s] += sv * ind; k += s
        acc[k] += ind
        iters.append(res.iters)
    return acc / float(len(iters)), iters


def realization_average(phases, lame, f, incl_phase=1, lam0=None, mu0=None, tol=1e-8, max_iter=10000,
                         solver=None):
    """Ensemble average over deterministic realisations (Sec. 3, Eq. 3.8):
    the force stays fixed and every microstructure ``X^j`` in ``phases`` (maps
    of one grid sharing the phase table ``lame``) is solved unshifted; ``u``,
    ``u V``, ``eps``, ``eps V``, ``sigma``, ``sigma V`` and ``V`` are summed
    over the realisations and divided by their number, in the component
    order of ``translate_average``.  The reference medium comes from the
    shared table unless given.  Returns ``[2d + 4s + 1][grid]`` and the
    per-realisation iteration counts."""
    phases = [np.asarray(ph) for ph in phases]
    shape = phases[0].shape
    d = len(shape)
    if lam0 is None or mu0 is None:
        lam0, mu0 = reference_medium(lame)
    solver = solver or solve_basic
    s = len(VOIGT[d])
    acc = np.zeros((2 * d + 4 * s + 1,) + shape)
    iters = []
    for ph in phases:
        if ph.shape != shape:
            raise ValueError("realisations must share one grid")
        res = solver(ph, lame, f, lam0, mu0, tol=tol, max_iter=max_iter)
        ind = (ph == incl_phase).astype(np.float64)
        ev, sv = to_voigt(res.eps), to_voigt(res.sig)
        k = 0
        acc[k:k + d] += res.u; k += d
        acc[k:k + d] += res.u * ind; k += d
        acc[k:k + s] += ev; k += s
        acc[k:k + s] += ev * ind; k += s
        acc[k:k + s] += sv; k += s
        acc[k:k + s] += sv * ind; k += s
        acc[k] += ind
        iters.append(res.iters)
    return acc / float(len(iters)), iters


def kernel_convolve(kernel, f):
    """Periodic convolution of a force with a kernel of the same grid
    (Sec. 6 dataset: the full-shift translated average of Eqs. 3.3-3.6 is
    the convolution of the force with the averaged point-force response):
    ``out_c = sum_j K_cj * P f_j`` with ``P`` the projection off the
    ``xi = 0`` set, written as the product of the transforms (Eqs. 4.3-4.5).
    ``kernel`` is ``[s][d][grid]``, ``f`` is ``[d][grid]``."""
    f = np.asarray(f, dtype=np.float64)
    shape = f.shape[1:]
    f_hat = fft_r(f, shape)
    f_hat[:, zero_set(shape)] = 0.0
    k_hat = fft_r(np.asarray(kernel, dtype=np.float64), shape)
    out_hat = np.stack([sum(k_hat[c, j] * f_hat[j] for j in range(f.shape[0])) for c in range(k_hat.shape[0])])
    return ifft_r(out_hat, shape)


def tensor_magnitude(tv):
    """``sqrt(sum_ab t_ab^2)`` of a Voigt field ``[s][grid]`` (tensor shear
    counted twice), summed component by component in Voigt order."""
    tv = np.asarray(tv, dtype=np.float64)
    d = 3 if tv.shape[0] == 6 else 2
    a = np.zeros(tv.shape[1:])
    for c in range(tv.shape[0]):
        q = tv[c] * tv[c]
        a = a + (q if c < d else 2.0 * q)
    return np.sqrt(a)


def radial_maxima(field, center, h=None, dr=1.0):
    """Largest value of ``field`` (a scalar ``[grid]``) per distance bin of
    width ``dr`` about ``center`` (array order, voxel units), distances
    measured to the nearest periodic image of the centre in the spacing
    ``h`` (array order).  Returns the maxima ``[nbins]``, nbins covering the
    half-diagonal of the cell."""
    field = np.asarray(field, dtype=np.float64)
    shape = field.shape
    d = len(shape)
    h = [1.0] * d if h is None else list(h)
    r2 = np.zeros(shape)
    half2 = 0.0
    # summed in the fixed order x, y, z: the rounding of the squared
    # distance decides the bin of a node that sits on a bin edge, so the
    # order is part of the definition (any fixed order is a valid reading)
    for a in reversed(range(d)):
        n = shape[a]
        idx = np.arange(n, dtype=np.float64) - float(center[a])
        img = idx - float(n) * np.rint(idx / float(n))
        off = img * h[a]
        shp = [1] * d
        shp[a] = n
        r2 = r2 + (off * off).reshape(shp)
        half2 += (0.5 * n * h[a]) ** 2
    nbins = int(np.floor(np.sqrt(half2) / dr)) + 1
    b = np.minimum(np.floor(np.sqrt(r2) / dr).astype(np.int64), nbins - 1)
    out = np.zeros(nbins)
    np.maximum.at(out, b.ravel(), field.ravel())
    return out


def rve_radius(avg, center, support_radius, tol, h=None, dr=1.0):
    """RVE of Definition 2.2 from averaged fields ``avg`` (the layout of
    ``translate_average``): the smallest bin edge beyond which the averaged
    strain and stress magnitudes both stay below ``tol`` times their maxima,
    and whether the annulus of width ``support_radius / 2`` around that ball
    (where the fields must stay stabilized) lies inside the periodic cell.
    Returns ``(radius, fits, maxima of |eps|, maxima of |sigma|)``."""
    avg = np.asarray(avg)
    shape = avg.shape[1:]
    d = len(shape)
    s = len(VOIGT[d])
    h = [1.0] * d if h is None else list(h)
    pe = radial_maxima(tensor_magnitude(avg[2 * d:2 * d + s]), center, h, dr)
    ps = radial_maxima(tensor_magnitude(avg[2 * d + 2 * s:2 * d + 3 * s]), center, h, dr)
    ge, gs = pe.max(), ps.max()
    first = len(pe)
    for b in range(len(pe) - 1, -1, -1):
        if pe[b] < tol * ge and ps[b] < tol * gs:
            first = b
        else:
            break
    if ge == 0.0 and gs == 0.0:
        first = 0
    radius = first * dr if first < len(pe) else np.inf
    box = min(0.5 * shape[a] * h[a] for a in range(d))
    fits = bool(np.isfinite(radius) and radius + 0.5 * support_radius <= box)
    return radius, fits, pe, ps


def relative_strain_error(eps, eps_ref):
    """``||eps - eps_ref||_F / ||eps_ref||_F`` over all voxels for full tensor
    fields ``[d][d][grid]``."""
    eps = np.asarray(eps, dtype=np.float64)
    ref = np.asarray(eps_ref, dtype=np.float64)
    return float(np.linalg.norm(eps - ref) / np.linalg.norm(ref))


def relative_strain_error_voigt(ev, ev_ref):
    """The same norm for Voigt fields ``[s][grid]`` (tensor shear, counted twice)."""
    ev = np.asarray(ev, dtype=np.float64)
    ref = np.asarray(ev_ref, dtype=np.float64)
    s = ev.shape[0]
    d = 2 if s == 3 else 3
    wts = np.array([1.0 if i == j else 2.0 for (i, j) in VOIGT[d]]).reshape((s,) + (1,) * (ev.ndim - 1))
    return float(np.sqrt(np.sum(wts * (ev - ref) ** 2) / np.sum(wts * ref ** 2)))
