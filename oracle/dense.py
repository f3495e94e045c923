"""Brute-force dense solve of the discrete BFCS equilibrium system.

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

The discrete problem of Eq. 5.5 (Sec. 5) is assembled here as an explicit
real matrix, without any FFT routine and without the iterative oracle's
operators: the spectral derivative along an axis is the circulant matrix
``D[a, b] = (1/N) sum_k i xi_k exp(2 pi i k (a - b) / N)`` written from the
DFT definition (Eqs. 4.3-4.5 with the derivative rule Eq. 4.8, Nyquist
wavevector read as 0); strain, Hooke's law and divergence are assembled as
Kronecker products and pointwise diagonals.  The system
``-div(L sym grad u) = P f`` is symmetric positive semi-definite with null
space the modes where the wavevector vanishes; its minimum-norm solution is
the limit every convergent scheme of the method reaches.  Sizes are limited
to a few hundred unknowns.
"""
from __future__ import annotations

import numpy as np


def derivative_matrix_1d(n: int) -> np.ndarray:
    """Real ``n x n`` spectral derivative matrix from the DFT definition."""
    k = np.arange(n)
    signed = np.where(k < n // 2, k, k - n).astype(np.float64)
    signed[n // 2] = 0.0                     # Nyquist wavevector read as zero
    xi = 2.0 * np.pi * signed / n
    a = np.arange(n).reshape(-1, 1)
    b = np.arange(n).reshape(1, -1)
    m = np.zeros((n, n), dtype=np.complex128)
    for kk in range(n):
        m += 1j * xi[kk] * np.exp(2j * np.pi * kk * (a - b) / n)
    m /= n
    return m.real


def zero_mode_projector(shape) -> np.ndarray:
    """``P = I - sum v v^T`` over the real unit modes whose wavevector is zero
    in every direction (index 0 or N/2 on each axis)."""
    d = len(shape)
    npts = int(np.prod(shape))
    p = np.eye(npts)
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    for corner in range(2 ** d):
        v = np.ones(shape)
        for a in range(d):
            if (corner >> a) & 1:
                v = v * np.cos(np.pi * grids[a])          # (-1)^n: the N/2 mode
        v = v.ravel() / np.sqrt(npts)
        p -= np.outer(v, v)
    return p


def axis_operator(shape, axis_array: int, m1d: np.ndarray) -> np.ndarray:
    """Apply a 1-D matrix along one array axis of a C-ordered flattened grid."""
    mats = [np.eye(n) for n in shape]
    mats[axis_array] = m1d
    out = mats[0]
    for m in mats[1:]:
        out = np.kron(out, m)
    return out


def assemble(phase, lame):
    """Return ``(A, D)``: the ``d npts`` square matrix of ``-div(L sym grad .)``
    and the list of derivative matrices, direction ``alpha = 0`` along x."""
    phase = np.asarray(phase)
    shape = phase.shape
    d = len(shape)
    npts = int(np.prod(shape))
    lame = np.asarray(lame, dtype=np.float64)
    lam = lame[phase.ravel(), 0]
    mu = lame[phase.ravel(), 1]
    D = [axis_operator(shape, d - 1 - alpha, derivative_matrix_1d(shape[d - 1 - alpha]))
         for alpha in range(d)]
    # strain operator: eps_ij = (D_i u_j + D_j u_i) / 2, block rows (i, j)
    S = np.zeros((d, d, npts, d * npts))
    for i in range(d):
        for j in range(d):
            S[i, j][:, j * npts:(j + 1) * npts] += 0.5 * D[i]
            S[i, j][:, i * npts:(i + 1) * npts] += 0.5 * D[j]
    # stress: sig_ij = lam tr(eps) delta_ij + 2 mu eps_ij (pointwise)
    tr = sum(S[i, i] for i in range(d))
    A = np.zeros((d * npts, d * npts))
    for i in range(d):
        row = np.zeros((npts, d * npts))
        for j in range(d):
            sig_ij = 2.0 * mu[:, None] * S[i, j]
            if i == j:
                sig_ij = sig_ij + lam[:, None] * tr
            row += D[j] @ sig_ij                      # (div sigma)_i
        A[i * npts:(i + 1) * npts] = -row
    return A, D


def dense_solve(phase, lame, f):
    """Minimum-norm solution of ``-div(L sym grad u) = P f``.

    Returns ``(u, eps, sig)`` as ``[d][grid]``, ``[d][d][grid]``, ``[d][d][grid]``.
    """
    phase = np.asarray(phase)
    shape = phase.shape
    d = len(shape)
    npts = int(np.prod(shape))
    A, D = assemble(phase, lame)
    P = zero_mode_projector(shape)
    rhs = np.concatenate([P @ np.asarray(f[c], dtype=np.float64).ravel() for c in range(d)])
    u = np.linalg.pinv(A, rcond=1e-12, hermitian=True) @ rhs
    uc = u.reshape(d, npts)
    lame = np.asarray(lame, dtype=np.float64)
    lam = lame[phase.ravel(), 0]
    mu = lame[phase.ravel(), 1]
    eps = np.zeros((d, d, npts))
    for i in range(d):
        for j in range(d):
            eps[i, j] = 0.5 * (D[i] @ uc[j] + D[j] @ uc[i])
    tr = sum(eps[i, i] for i in range(d))
    sig = 2.0 * mu * eps
    for i in range(d):
        sig[i, i] += lam * tr
    return (uc.reshape((d,) + shape), eps.reshape((d, d) + shape), sig.reshape((d, d) + shape))
