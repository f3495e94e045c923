"""The nonlocal kernel surrogate of Sec. 6 (Eqs. 6.5-6.6) for the averaged
displacement, around the library's nonlocal kernels.

The operator maps an averaged displacement field to
``L_c[u](x) = sum over grid offsets 0 < |r| < delta of K_c(|r|) (u(x + r) - u(x))``
with a radial scalar kernel in the Bernstein basis of degree M on
[0, delta], acting on each component alike; for the displacement type the
response it must reproduce is the negated body force, ``Gamma_k = -b_k``.
The fit of Eq. 6.6 (least squares plus a Tikhonov term lam ||c||^2) is a
quadratic in the M + 1 coefficients: the library assembles its normal
equations on the device in FP64 and solves them in closed form or runs the
paper's optimiser, Adam, on the same loss.

Dataset: for one periodic microstructure the translated average over every
shift of a cell is the convolution of the force with the averaged response
to a point force, so ``<u>_k`` comes from one library convolution per force
with the averaged displacement kernel (``surrogate.averaged_kernels``).
Torch holds device memory only; every arithmetic step runs in the library.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .lsfft import (Plan, block_mean, nonlocal_apply, nonlocal_fit, nonlocal_normal_equations, sample_norms)
from .surrogate import averaged_displacement_from_kernel


def pairs(Ku, forces, plan: Plan | None = None):
    """(<u>_k, Gamma_k = -b_k) for forces ``[B][3][...grid]`` (the kernel's
    dtype): the averaged displacement by the kernel convolution and the
    negated force (a library scaled copy)."""
    u = averaged_displacement_from_kernel(Ku, forces, plan=plan)
    return u, block_mean(forces.contiguous(), 1, scale=-1.0, spatial=forces.dim() - 2)


class NormalEquations:
    """Running sums of the normal equations over batches of pairs."""

    def __init__(self, degree: int, delta: float):
        self.degree, self.delta = int(degree), float(delta)
        self.G = np.zeros((degree + 1, degree + 1))
        self.g = np.zeros(degree + 1)
        self.gg = 0.0
        self.count = 0

    def add(self, u, gamma):
        G, g, gg = nonlocal_normal_equations(u.contiguous(), gamma.contiguous(), self.degree, self.delta)
        self.G += G
        self.g += g
        self.gg += gg
        self.count += int(u.shape[0])
        return self

    def loss(self, c, lam: float = 0.0) -> float:
        c = np.asarray(c, dtype=np.float64)
        return float(c @ self.G @ c - 2.0 * self.g @ c + self.gg + lam * c @ c)


@dataclass
class NonlocalOperator:
    """A fitted operator L_c with its horizon."""
    c: np.ndarray
    delta: float

    @property
    def degree(self) -> int:
        return len(self.c) - 1

    def apply(self, u):
        """L_c[u] of fields ``[B][d][...grid]``."""
        return nonlocal_apply(u.contiguous(), self.c, self.delta)

    def kernel(self, rho):
        """K_c(rho) (zero from the horizon on), for inspection."""
        from math import comb
        t = np.asarray(rho, dtype=np.float64) / self.delta
        M = self.degree
        k = sum(self.c[m] * comb(M, m) * t ** m * (1.0 - t) ** (M - m) for m in range(M + 1))
        return np.where((t > 0) & (t < 1), k, 0.0)

    def relative_residual(self, u, gamma):
        """Per-sample ||L_c[u] - Gamma|| / ||Gamma|| (FP64 numpy)."""
        nd, nt = sample_norms(gamma.contiguous(), self.apply(u))
        return nd / nt


def fit(ne: NormalEquations, lam: float, adam_steps: int = 0, lr: float = 1e-3) -> NonlocalOperator:
    """Eq. 6.6 from accumulated normal equations: the closed-form minimiser
    (``adam_steps = 0``) or Adam from zero.  Adam runs on the loss divided by
    trace(G) / (M + 1), which has the same minimiser and unit-scale
    curvature, so one step size serves any data scale."""
    if adam_steps == 0:
        c = nonlocal_fit(ne.G, ne.g, lam)
    else:
        s = float(np.trace(ne.G)) / (ne.degree + 1)
        if not s > 0.0:
            raise ValueError("the normal equations are empty")
        c = nonlocal_fit(ne.G / s, ne.g / s, lam / s, adam_steps=adam_steps, lr=lr)
    return NonlocalOperator(c, ne.delta)
