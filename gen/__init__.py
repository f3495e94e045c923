"""Seeded synthetic inputs for the BFCS Lippmann-Schwinger solver and its oracle.

This module only *generates inputs*: phase maps of periodic microstructures,
compactly supported body-force fields, material tables given as Young's
modulus and Poisson's ratio, and translation sets.  It holds none of the
solver's arithmetic (no Lame conversion, no Green operator, no transform), so
the oracle and the GPU path can both draw from it without sharing method code.

Conventions shared by every generator here:

* A grid is given in array order: ``(ny, nx)`` in 2D, ``(nz, ny, nx)`` in 3D.
  Node ``k`` sits at position ``k * h`` with ``h = 1`` voxel (Sec. 4, Eq. 4.1).
* Vector fields are component-major ``[d][...grid]``, component 0 along x.
* Phase maps are ``uint8`` with phase 0 the matrix and phase 1 the inclusions.
* All randomness comes from ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Material", "inclusion_per_cell", "rsa_cell", "tile_cell", "laminate",
    "bump_force", "dipole_force", "multi_bump_force", "sample_shifts",
    "all_shifts", "random_direction", "random_center", "grid_positions",
    "bump_set_params", "point_force",
]


@dataclass(frozen=True)
class Material:
    """Isotropic phases by Young's modulus and Poisson's ratio, phase id = index."""

    young: tuple
    poisson: tuple

    def table(self) -> np.ndarray:
        """``[nphase][2]`` array of ``(E, nu)``."""
        return np.array(list(zip(self.young, self.poisson)), dtype=np.float64)

    @staticmethod
    def two_phase(e_matrix: float, e_incl: float, nu: float = 0.3) -> "Material":
        return Material(young=(float(e_matrix), float(e_incl)), poisson=(nu, nu))


def grid_positions(shape):
    """Integer node coordinates per axis in array order, broadcastable to ``shape``."""
    d = len(shape)
    out = []
    for a, n in enumerate(shape):
        s = [1] * d
        s[a] = n
        out.append(np.arange(n).reshape(s))
    return out


def _periodic_offset(pos, c, period):
    """Minimum-image signed offset ``pos - c`` on a ring of length ``period``."""
    t = (pos - c) % period
    return np.where(t > period / 2.0, t - period, t)


def _cell_ball_mask(cell_shape, center, radius):
    pos = grid_positions(cell_shape)
    r2 = 0.0
    for a, n in enumerate(cell_shape):
        off = _periodic_offset(pos[a].astype(np.float64), center[a], n)
        r2 = r2 + off * off
    return r2 <= radius * radius


def inclusion_per_cell(shape, cell: int, vf: float) -> tuple[np.ndarray, float]:
    """One centred disk/sphere per ``cell^d`` unit cell, tiled over ``shape``.

    The radius is chosen so the voxel count in a cell is the one nearest
    ``vf * cell^d``; a node belongs to the inclusion when it lies inside the
    ball centred at ``(cell - 1) / 2`` per axis.  Returns the phase map and
    the achieved volume fraction.
    """
    d = len(shape)
    for n in shape:
        if n % cell:
            raise ValueError("grid must hold a whole number of cells")
    cshape = (cell,) * d
    center = [(cell - 1) / 2.0] * d
    pos = grid_positions(cshape)
    r2 = sum((pos[a] - center[a]) ** 2 for a in range(d))
    target = vf * cell ** d
    radii = np.unique(np.sqrt(r2.ravel()))
    counts = np.array([(r2 <= r * r + 1e-9).sum() for r in radii])
    best = radii[int(np.argmin(np.abs(counts - target)))]
    mask = (r2 <= best * best + 1e-9)
    phase_cell = mask.astype(np.uint8)
    return tile_cell(phase_cell, shape), float(phase_cell.mean())


def rsa_cell(cell: int, d: int, vf: float, rmin: float, rmax: float, seed: int,
             max_fail: int = 2000, max_restart: int = 200) -> tuple[np.ndarray, float]:
    """Random non-overlapping balls in one periodic ``cell^d`` cell (seeded RSA).

    Centres are uniform in the cell, radii uniform in ``[rmin, rmax]``; a new
    ball is kept when its periodic minimum-image distance to every kept ball
    exceeds the sum of radii.  Balls are added until the voxelised volume
    fraction reaches ``vf``; after ``max_fail`` rejections in a row the cell
    restarts.  Returns the cell phase map and the achieved volume fraction.
    """
    rng = np.random.default_rng(seed)
    cshape = (cell,) * d
    for _ in range(max_restart):
        balls = []
        mask = np.zeros(cshape, dtype=bool)
        fails = 0
        while mask.mean() < vf and fails < max_fail:
            c = rng.uniform(0.0, cell, size=d)
            r = rng.uniform(rmin, rmax)
            ok = True
            for (c2, r2) in balls:
                off = _periodic_offset(c, c2, cell)
                if math.sqrt(float((off * off).sum())) <= r + r2:
                    ok = False
                    break
            if not ok:
                fails += 1
                continue
            trial = mask | _cell_ball_mask(cshape, c, r)
            if trial.mean() > vf + 0.5 * (trial.mean() - mask.mean()) and balls:
                # overshoot by more than half of this ball: try a smaller one
                fails += 1
                continue
            fails = 0
            balls.append((c, r))
            mask = trial
        if mask.mean() >= vf - 0.02:
            return mask.astype(np.uint8), float(mask.mean())
    raise RuntimeError("RSA could not reach the requested volume fraction")


def tile_cell(phase_cell: np.ndarray, shape) -> np.ndarray:
    """Periodic tiling of one cell over a grid of whole cells."""
    reps = tuple(n // c for n, c in zip(shape, phase_cell.shape))
    return np.ascontiguousarray(np.tile(phase_cell, reps)).astype(np.uint8)


def laminate(shape, widths, axis_x: bool = True) -> np.ndarray:
    """Layers normal to x, alternating phases 0,1,0,1,... with the given widths.

    ``sum(widths)`` must divide ``nx``; the stack repeats along x.
    """
    nx = shape[-1]
    period = int(sum(widths))
    if nx % period:
        raise ValueError("layer period must divide nx")
    row = np.concatenate([np.full(w, i % 2, dtype=np.uint8) for i, w in enumerate(widths)])
    row = np.tile(row, nx // period)
    return np.ascontiguousarray(np.broadcast_to(row, shape)).astype(np.uint8)


def random_center(shape, seed: int) -> np.ndarray:
    """Continuous seeded point in the grid box, array-order coordinates."""
    rng = np.random.default_rng(seed)
    return np.array([rng.uniform(0.0, n) for n in shape])


def random_direction(d: int, seed: int) -> np.ndarray:
    """Seeded unit vector uniform on the circle/sphere, component 0 along x."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=d)
    return v / np.linalg.norm(v)


def _bump(shape, center, radius):
    """``exp(-1/(1 - r^2/R^2))`` inside ``r < R`` (periodic minimum image), else 0."""
    pos = grid_positions(shape)
    r2 = 0.0
    for a, n in enumerate(shape):
        off = _periodic_offset(pos[a].astype(np.float64), center[a], n)
        r2 = r2 + off * off
    q = r2 / (radius * radius)
    out = np.zeros(np.broadcast_shapes(*[p.shape for p in pos]), dtype=np.float64)
    inside = q < 1.0
    out[inside] = np.exp(-1.0 / (1.0 - q[inside]))
    return out


def bump_force(shape, center, radius: float, direction) -> np.ndarray:
    """Vector bump force ``f = bump(x) * direction`` of amplitude 1 (peak 1/e).

    ``center`` is in array order; ``direction`` is component-major (x first).
    Returns ``[d][...shape]`` float64.
    """
    b = _bump(shape, center, radius)
    direction = np.asarray(direction, dtype=np.float64)
    return np.stack([b * direction[c] for c in range(len(shape))])


def dipole_force(shape, center, radius: float, direction, sep: int) -> np.ndarray:
    """Self-equilibrated pair ``bump(x - a) e - bump(x + a) e``, ``a`` integer along x.

    Both bumps are the same sampled profile shifted by whole voxels, so the
    grid sum of the force is exactly zero.
    """
    b = _bump(shape, center, radius)
    shift = int(sep)
    pair = np.roll(b, shift, axis=-1) - np.roll(b, -shift, axis=-1)
    direction = np.asarray(direction, dtype=np.float64)
    return np.stack([pair * direction[c] for c in range(len(shape))])


def multi_bump_force(shape, seed: int, nmin: int = 1, nmax: int = 3,
                     rmin: float = 4.0, rmax: float = 12.0) -> np.ndarray:
    """Sum of 1-3 seeded vector bumps with random centres, radii and directions."""
    rng = np.random.default_rng(seed)
    d = len(shape)
    k = int(rng.integers(nmin, nmax + 1))
    out = np.zeros((d,) + tuple(shape))
    for _ in range(k):
        c = np.array([rng.uniform(0.0, n) for n in shape])
        r = rng.uniform(rmin, rmax)
        v = rng.normal(size=d)
        v /= np.linalg.norm(v)
        out += bump_force(shape, c, r, v)
    return out


def all_shifts(cell: int, d: int) -> np.ndarray:
    """Every integer translation inside one ``cell^d`` cell, ``[n][d]`` in array order."""
    g = np.stack(np.meshgrid(*([np.arange(cell)] * d), indexing="ij"), axis=-1)
    return g.reshape(-1, d).astype(np.int32)


def sample_shifts(cell: int, d: int, n: int, seed: int) -> np.ndarray:
    """Seeded subset (without replacement) of the intra-cell translations."""
    full = all_shifts(cell, d)
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(len(full), size=n, replace=False))
    return np.ascontiguousarray(full[idx])


def point_force(shape, direction_index: int) -> np.ndarray:
    """Unit force at the origin voxel along one axis (component-major)."""
    f = np.zeros((len(shape),) + tuple(shape))
    f[(direction_index,) + (0,) * len(shape)] = 1.0
    return f


def bump_set_params(n: int, count: int, seed: int, nmin: int = 1, nmax: int = 3,
                    rmin: float = 4.0, rmax: float = 12.0) -> list:
    """Seeded parameters of ``count`` forces on an ``n^3`` grid, each a sum of
    ``nmin..nmax`` vector bumps with uniform centres, radii uniform in
    ``[rmin, rmax]`` and directions uniform on the sphere.  Returns a list of
    lists of ``(center[3] array order, radius, direction[3] x first)``."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        k = int(rng.integers(nmin, nmax + 1))
        bumps = []
        for _ in range(k):
            c = rng.uniform(0.0, n, size=3)
            r = float(rng.uniform(rmin, rmax))
            v = rng.normal(size=3)
            bumps.append((c, r, v / np.linalg.norm(v)))
        out.append(bumps)
    return out


