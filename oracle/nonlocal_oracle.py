"""Plain float64 NumPy oracle of the nonlocal kernel surrogate of Sec. 6
(Eqs. 6.5-6.6).

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

The operator of Eq. 6.5 maps an averaged displacement field to
``L_c[u](x) = sum_{0 < |r| < delta} K_c(|r|) (u(x + r) - u(x)) h^d`` on the
periodic grid (the integral over y written as a sum over grid offsets
r = y - x, h = 1), with a radial kernel expanded in the Bernstein basis of
degree M on [0, delta]:

    K_c(rho) = sum_m c_m B_{m,M}(rho / delta),
    B_{m,M}(t) = binom(M, m) t^m (1 - t)^(M - m),

and K = 0 for rho >= delta.  It acts on every displacement component alike
(``form = 0``, the literal reading).  With ``form = 1`` the kernel is the
isotropic matrix function of the bond r = y - x,

    K(r) = K1(|r|) I + K2(|r|) e e^T,   e = r / |r| (components x first),

each of K1, K2 expanded in the same basis: coefficients (c1_0..c1_M,
c2_0..c2_M).  Eq. 6.7 pairs the stress-type kernel with the bond vector,
so the paper's kernels are tensors of the bond; this is the general such
kernel for the displacement type, and the term e e^T couples the components
as the divergence term of an isotropic Navier operator does.
Eq. 6.6 fits the coefficients to pairs (<u>_k, Gamma_k) with Gamma_k = -b_k
(the operator type of the body force):

    c* = argmin_c  sum_k || L_c[<u>_k] - Gamma_k ||^2 + lam ||c||^2

(Tikhonov term on the coefficients).  The loss is quadratic in c: with the
features Phi_m[u] = sum_r B_m(|r| / delta) (u(x + r) - u(x)), the normal
equations are (G + lam I) c = g, G_mn = sum_k <Phi_m[u_k], Phi_n[u_k]>,
g_m = sum_k <Phi_m[u_k], Gamma_k>.  The paper fits with Adam; ``fit_adam``
does that on the same quadratic, ``fit_closed`` solves the normal
equations.  Readings: the kernel is scalar and acts componentwise; r runs
over grid offsets strictly inside the horizon; lam multiplies the plain
Euclidean norm of c.
"""
from __future__ import annotations

from math import comb

import numpy as np


def bernstein(M: int, t):
    """``[M + 1][...]``: B_{m,M}(t) for m = 0..M."""
    t = np.asarray(t, dtype=np.float64)
    return np.stack([comb(M, m) * t ** m * (1.0 - t) ** (M - m) for m in range(M + 1)])


def ball_offsets(d: int, delta: float):
    """Integer offsets r with 0 < |r| < delta in d dimensions, and |r|."""
    R = int(np.ceil(delta))
    rng = np.arange(-R, R + 1)
    grids = np.meshgrid(*([rng] * d), indexing="ij")
    offs = np.stack([g.ravel() for g in grids], axis=1)
    rho = np.sqrt((offs.astype(np.float64) ** 2).sum(axis=1))
    keep = (rho > 0.0) & (rho < delta)
    return offs[keep], rho[keep]


def features(u, M: int, delta: float, form: int = 0):
    """Phi_m[u] for m = 0..M, ``[M + 1][comp][grid]``: the sum over the
    horizon's offsets of B_m(|r| / delta) (u(x + r) - u(x)).  With
    ``form = 1`` also the features of the e e^T term,
    sum_r B_m(|r| / delta) e (e . (u(x + r) - u(x))), after them:
    ``[2 (M + 1)][comp][grid]``.  Offsets are in array order (z first in
    3D); the direction e is taken in component order (x first)."""
    u = np.asarray(u, dtype=np.float64)
    d = u.ndim - 1
    offs, rho = ball_offsets(d, delta)
    w = bernstein(M, rho / delta)                 # [M + 1][noffsets]
    out = np.zeros(((2 if form == 1 else 1) * (M + 1),) + u.shape)
    axes = tuple(range(1, d + 1))
    for i, r in enumerate(offs):
        diff = np.roll(u, shift=tuple(-int(v) for v in r), axis=axes) - u      # u(x + r) - u(x)
        for m in range(M + 1):
            out[m] += w[m, i] * diff
        if form == 1:
            e = r[::-1].astype(np.float64) / rho[i]                           # x first
            proj = np.tensordot(e, diff, axes=(0, 0))                           # e . (u(x + r) - u(x))
            for m in range(M + 1):
                out[M + 1 + m] += w[m, i] * e.reshape((d,) + (1,) * d) * proj
    return out


def apply_operator(c, u, delta: float, form: int = 0):
    """L_c[u] of Eq. 6.5 for coefficients ``c`` (degree len(c) - 1, or
    len(c) / 2 - 1 with ``form = 1``)."""
    c = np.asarray(c, dtype=np.float64)
    M = (len(c) // 2 if form == 1 else len(c)) - 1
    return np.tensordot(c, features(u, M, delta, form), axes=(0, 0))


def normal_equations(us, gammas, M: int, delta: float, form: int = 0):
    """G and g of the quadratic loss over the pairs (u_k, Gamma_k), and
    sum_k ||Gamma_k||^2."""
    nf = (2 if form == 1 else 1) * (M + 1)
    G = np.zeros((nf, nf))
    g = np.zeros(nf)
    gg = 0.0
    for u, gam in zip(us, gammas):
        phi = features(u, M, delta, form).reshape(nf, -1)
        gam = np.asarray(gam, dtype=np.float64).ravel()
        G += phi @ phi.T
        g += phi @ gam
        gg += float(gam @ gam)
    return G, g, gg


def loss(c, G, g, gg, lam):
    """sum_k ||L_c[u_k] - Gamma_k||^2 + lam ||c||^2 from the normal equations."""
    c = np.asarray(c, dtype=np.float64)
    return float(c @ G @ c - 2.0 * g @ c + gg + lam * c @ c)


def fit_closed(G, g, lam):
    """The minimiser of Eq. 6.6: (G + lam I) c = g."""
    return np.linalg.solve(G + lam * np.eye(len(g)), g)


def fit_adam(G, g, lam, steps: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-12, c0=None):
    """Eq. 6.6 minimised by Adam (Kingma and Ba) on the quadratic: gradient
    2 (G c - g) + 2 lam c, bias-corrected moments, ``steps`` steps of size
    ``lr``, starting at ``c0`` (zero by default)."""
    c = np.zeros(len(g)) if c0 is None else np.array(c0, dtype=np.float64)
    m = np.zeros_like(c)
    v = np.zeros_like(c)
    for k in range(1, steps + 1):
        grad = 2.0 * (G @ c - g) + 2.0 * lam * c
        m = beta1 * m + (1.0 - beta1) * grad
        v = beta2 * v + (1.0 - beta2) * grad * grad
        c = c - lr * (m / (1.0 - beta1 ** k)) / (np.sqrt(v / (1.0 - beta2 ** k)) + eps)
    return c
