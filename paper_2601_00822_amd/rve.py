"""RVE identification and the body-force unit cell (Sec. 3, Definition 2.2).

The RVE is the ball about the centre of a self-equilibrated body force with
compact support outside which the averaged strain and stress vanish to a
relative tolerance; the fields must also stay stabilized over an annulus of
half the support's radius around it.  When that annulus does not fit in the
body-force unit cell (BFUC), the cell is enlarged and the averages are
solved again.  The radial profile and the radius come from the library
(``lsfft_rve_identify``); this module only drives the enlargement loop.
"""
from __future__ import annotations

import numpy as np

from .lsfft import Plan

# transform lengths the library accepts (products of 2 and 3 from 4 to 256)
LENGTHS = (4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 256)


def find_bfuc(cell_phase, lame, force_at, support_radius, shifts, tol=1e-2, cells=1, max_len=256, prec="f64",
              solve_tol=1e-8, max_batch=64, device="cuda", printer=None):
    """Smallest BFUC of ``k`` periodic cells per axis (k = cells, cells + 1,
    ... with k * cell a supported length up to max_len) whose RVE, plus half
    the support radius, fits inside it.

    ``cell_phase``: the periodic cell's phase map (array order);
    ``force_at(shape, center)``: the force ``[d][shape]`` (numpy, FP64) with
    its support centred at ``center`` (array order, voxel units);
    ``shifts``: translations of the averages (Eqs. 3.3-3.6), array order.
    Returns a dict with ``found``, ``shape``, the last RVE result ``rve``, its
    FP64 averages ``avg`` and the ``history`` of (shape, RVE result)."""
    import torch
    cell_phase = np.asarray(cell_phase, dtype=np.uint8)
    d = cell_phase.ndim
    history = []
    k = max(1, int(cells))
    while True:
        shape = tuple(k * n for n in cell_phase.shape)
        if max(shape) > max_len:
            return dict(found=False, shape=None, rve=None, avg=None, history=history)
        if any(n not in LENGTHS for n in shape):
            k += 1
            continue
        center = tuple(0.5 * n for n in shape)
        phase = np.ascontiguousarray(np.tile(cell_phase, (k,) * d))
        f = np.asarray(force_at(shape, center), dtype=np.float64)
        dt = torch.float64 if prec == "f64" else torch.float32
        plan = Plan([shape], prec=prec, max_batch=max_batch, refine=(prec == "f32"))
        try:
            avg, _ = plan.translate_average(torch.from_numpy(phase).to(device), lame,
                                            torch.from_numpy(f).to(device).to(dt), shifts, tol=solve_tol)
            info = plan.rve_identify(avg, center, support_radius, tol=tol)
        finally:
            plan.close()
        history.append((shape, info))
        if printer:
            printer(f"BFUC {shape}: RVE radius {info['radius']:.1f}, cell radius {info['box_radius']:.1f}, "
                    f"fits {info['fits']}")
        if info["fits"]:
            return dict(found=True, shape=shape, rve=info, avg=avg, history=history)
        k += 1
