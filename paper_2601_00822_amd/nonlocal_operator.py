"""The nonlocal kernel surrogate of Sec. 6 (Eqs. 6.5-6.6) for the averaged
displacement, around the library's nonlocal kernels.

The operator maps an averaged displacement field to
``L_c[u](x) = sum over grid offsets 0 < |r| < delta of K(r) (u(x + r) - u(x))``
with kernels in the Bernstein basis of degree M on [0, delta]: a radial
scalar K1(|r|) acting on each component alike (form 0), or the isotropic
matrix kernel K1(|r|) I + K2(|r|) e e^T of the bond direction e (form 1),
which couples the components.  For the displacement type the response it
must reproduce is the negated body force, ``Gamma_k = -b_k``.  The fit of
Eq. 6.6 (least squares plus a Tikhonov term lam ||c||^2) is a quadratic in
the (form + 1)(M + 1) coefficients: the library assembles its normal
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
    """Running sums of the normal equations over batches of pairs; ``form``
    0 is the scalar kernel, 1 the matrix kernel K1 I + K2 e e^T."""

    def __init__(self, degree: int, delta: float, form: int = 0):
        self.degree, self.delta, self.form = int(degree), float(delta), int(form)
        nf = (self.form + 1) * (self.degree + 1)
        self.G = np.zeros((nf, nf))
        self.g = np.zeros(nf)
        self.gg = 0.0
        self.count = 0

    def add(self, u, gamma):
        G, g, gg = nonlocal_normal_equations(u.contiguous(), gamma.contiguous(), self.degree, self.delta, self.form)
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
    """A fitted operator L_c with its horizon and kernel form."""
    c: np.ndarray
    delta: float
    form: int = 0

    @property
    def degree(self) -> int:
        return len(self.c) // (self.form + 1) - 1

    def apply(self, u):
        """L_c[u] of fields ``[B][d][...grid]``."""
        return nonlocal_apply(u.contiguous(), self.c, self.delta, self.form)

    def kernel(self, rho):
        """(K1(rho)[, K2(rho)]) (zero from the horizon on), for inspection."""
        from math import comb
        t = np.asarray(rho, dtype=np.float64) / self.delta
        M = self.degree
        out = []
        for f in range(self.form + 1):
            c = self.c[f * (M + 1):(f + 1) * (M + 1)]
            k = sum(c[m] * comb(M, m) * t ** m * (1.0 - t) ** (M - m) for m in range(M + 1))
            out.append(np.where((t > 0) & (t < 1), k, 0.0))
        return tuple(out)

    def long_wave_stiffness(self):
        """(C11, C12, C44): the cubic stiffness of the Navier operator the
        fitted 3D operator reduces to at long wavelengths.  With
        u(x + r) - u(x) expanded to second order, L_c[u]_a becomes
        sum_{b,i,j} (alpha d_ab d_ij + B_abij) d_i d_j u_b, alpha = 1/2
        sum_r K1 |r|^2 e_1^2 and B_abij = 1/2 sum_r K2 |r|^2 e_a e_b e_i e_j
        over the grid offsets inside the horizon (cubic symmetry of the
        lattice); matched to div(C grad u): C11 = alpha + B_1111,
        C44 = alpha + B_1122, C12 = 2 B_1212 - C44.  The analogue, for the
        displacement type, of the stiffness the paper takes from the
        stress-type kernel (Eq. 6.7).  Host arithmetic over the offsets."""
        from math import comb
        R = int(np.ceil(self.delta)) - 1
        g = np.arange(-R, R + 1)
        r = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3).astype(np.float64)
        rho = np.sqrt((r * r).sum(axis=1))
        keep = (rho > 0.0) & (rho < self.delta)
        r, rho = r[keep], rho[keep]
        e = r / rho[:, None]
        M = self.degree
        t = rho / self.delta
        basis = np.stack([comb(M, m) * t ** m * (1.0 - t) ** (M - m) for m in range(M + 1)])
        k1 = self.c[:M + 1] @ basis
        k2 = self.c[M + 1:] @ basis if self.form == 1 else np.zeros_like(k1)
        w1, w2 = 0.5 * k1 * rho ** 2, 0.5 * k2 * rho ** 2
        alpha = float(np.sum(w1 * e[:, 0] ** 2))
        b1111 = float(np.sum(w2 * e[:, 0] ** 4))
        b1122 = float(np.sum(w2 * e[:, 0] ** 2 * e[:, 1] ** 2))
        c44 = alpha + b1122
        return alpha + b1111, 2.0 * b1122 - c44, c44

    def relative_residual(self, u, gamma, equilibrated: bool = False):
        """Per-sample ||L_c[u] - Gamma|| / ||Gamma|| (FP64 numpy).  With
        ``equilibrated`` both norms leave out Gamma's mean (its part on the
        xi = 0 set, which no operator of this form produces: L_c[u] has zero
        mean, so ||L_c[u] - Gamma||^2 = ||L_c[u] - P Gamma||^2 + N |mean|^2);
        the means come from the library's block mean over the whole grid, so
        every grid axis must share one length."""
        nd, nt = sample_norms(gamma.contiguous(), self.apply(u))
        if not equilibrated:
            return nd / nt
        sp = tuple(gamma.shape[2:])
        if len(set(sp)) != 1:
            raise ValueError("the equilibrated residual needs equal grid lengths")
        mean = block_mean(gamma.contiguous(), sp[0], spatial=len(sp)).double().cpu().numpy()
        rm2 = float(np.prod(sp)) * (mean.reshape(mean.shape[0], -1) ** 2).sum(axis=1)
        return np.sqrt(np.maximum(nd ** 2 - rm2, 0.0) / np.maximum(nt ** 2 - rm2, 1e-300))


def fit(ne: NormalEquations, lam: float, adam_steps: int = 0, lr: float = 1e-3) -> NonlocalOperator:
    """Eq. 6.6 from accumulated normal equations: the closed-form minimiser
    (``adam_steps = 0``) or Adam from zero.  Adam runs on the loss divided by
    trace(G) / nc (nc coefficients), which has the same minimiser and
    unit-scale curvature, so one step size serves any data scale."""
    if adam_steps == 0:
        c = nonlocal_fit(ne.G, ne.g, lam)
    else:
        s = float(np.trace(ne.G)) / len(ne.g)
        if not s > 0.0:
            raise ValueError("the normal equations are empty")
        c = nonlocal_fit(ne.G / s, ne.g / s, lam / s, adam_steps=adam_steps, lr=lr)
    return NonlocalOperator(c, ne.delta, ne.form)
