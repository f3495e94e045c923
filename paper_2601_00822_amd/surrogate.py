"""Dataset, training and evaluation of the learned surrogate (Sec. 6, Fig. 5
blocks 2-3) around the HIP solver and the HIP surrogate kernels.

Dataset (the compressed dataset of Eq. 3.7 for one periodic
microstructure): the translation average over every shift of one cell is a
linear map of the force that commutes with grid translations, i.e. a
periodic convolution.  Its kernel, the averaged strain response to a unit
point force at the origin along each axis, comes from three
``translate_average`` calls of the batched solver (3 x cell^3 solves).  The
averaged strain of any force is then that kernel convolved with the force,
computed by the library's own transforms (``lsfft_kernel_convolve``); forces
and targets are restricted to the coarse grid by the library's block means.

Training and inference run entirely in the surrogate kernels (bf16 MFMA,
fp32 accumulation, Adam); this module only moves batches and schedules the
learning rate.  The solver supplies the held-out targets the surrogate is
measured against and stays the fallback: ``averaged_strain`` serves a
prediction only when its error, judged per input against the exact
averaged kernel, is within the caller's bound.  Torch holds the device
memory; every arithmetic step runs in the library.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from .fno import FnoArch, Surrogate, pack
from .lsfft import Plan, block_mean, relative_l2 as _relative_l2


def cell_shifts(cell: int, d: int = 3) -> np.ndarray:
    """Every integer shift inside one cell, ``[cell^d][d]`` in array order."""
    g = np.stack(np.meshgrid(*([np.arange(cell)] * d), indexing="ij"), axis=-1)
    return g.reshape(-1, d).astype(np.int32)


def averaged_kernels(phase, lame, cell: int, prec: str = "f64", max_batch: int = 512, tol: float = 1e-8):
    """The averaged responses to a unit point force at the origin along each
    axis j (x first): ``K[c][j]`` for the strain components c (Voigt) and
    ``Ku[a][j]`` for the displacement components a, from three
    ``translate_average`` calls over every shift of one cell.  FP64 (or
    FP32) torch tensors ``[6][3][n][n][n]`` and ``[3][3][n][n][n]``, and the
    per-shift reports."""
    import torch
    shape = tuple(phase.shape)
    d = len(shape)
    if d != 3:
        raise ValueError("the surrogate dataset is 3D")
    plan = Plan([shape], prec=prec, max_batch=max_batch, refine=(prec == "f32"))
    dt = torch.float64 if prec == "f64" else torch.float32
    shifts = cell_shifts(cell, d)
    cols, ucols, reps = [], [], []
    try:
        for j in range(d):
            f = torch.zeros((d,) + shape, dtype=dt, device=phase.device)
            f[(j,) + (0,) * d] = 1.0
            avg, r = plan.translate_average(phase, lame, f, shifts, tol=tol)
            cols.append(avg[2 * d:2 * d + 6].clone())
            ucols.append(avg[0:d].clone())
            reps += r
    finally:
        plan.close()
    return torch.stack(cols, dim=1), torch.stack(ucols, dim=1), reps


def averaged_strain_kernel(phase, lame, cell: int, prec: str = "f64", max_batch: int = 512, tol: float = 1e-8):
    """``K[c][j]`` = the translation-averaged strain component ``c`` (Voigt)
    for a unit point force along axis ``j`` (x first) at the origin; FP64
    torch tensor ``[6][3][n][n][n]``.  Returns (K, per-shift reports)."""
    K, _, reps = averaged_kernels(phase, lame, cell, prec=prec, max_batch=max_batch, tol=tol)
    return K, reps


def averaged_strain_from_kernel(K, f, plan: Plan | None = None, max_batch: int = 64):
    """``f`` [B][3][n][n][n] -> averaged strain [B][6][n][n][n]: the
    convolution with the averaged kernel ``K`` [6][3][n][n][n], by the
    library in the kernel's precision (a plan of that grid may be passed in
    to reuse its workspace)."""
    shape = tuple(K.shape[-3:])
    own = plan is None
    if own:
        import torch
        plan = Plan([shape], prec="f64" if K.dtype == torch.float64 else "f32", max_batch=max_batch)
    try:
        return plan.kernel_convolve(K.contiguous(), f.contiguous())
    finally:
        if own:
            plan.close()


def averaged_displacement_from_kernel(Ku, f, plan: Plan | None = None, max_batch: int = 64):
    """``f`` [B][3][n][n][n] -> averaged displacement [B][3][n][n][n]: the
    convolution with the averaged displacement kernel ``Ku`` [3][3][...]
    (given to the library as the first rows of a six-row kernel)."""
    import torch
    d = Ku.shape[0]
    K6 = torch.zeros((6,) + tuple(Ku.shape[1:]), dtype=Ku.dtype, device=Ku.device)
    K6[:d] = Ku
    return averaged_strain_from_kernel(K6, f, plan=plan, max_batch=max_batch)[:, :d].contiguous()


def restrict2(a, dtype=None, scale: float = 1.0):
    """2 x 2 x 2 block means of the last three axes (times ``scale``, as
    ``dtype``), by the library."""
    return block_mean(a.contiguous(), 2, scale=scale, dtype=dtype)


def init_params(arch: FnoArch, seed: int) -> np.ndarray:
    """Seeded initial parameters: pointwise weights uniform in
    ``+-1/sqrt(fan_in)``, zero biases, spectral weights with real and
    imaginary parts uniform in ``+-1/width``."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in arch.layout():
        if name.startswith("r"):
            s = 1.0 / arch.width
            p[name] = rng.uniform(-s, s, size=shp) + 1j * rng.uniform(-s, s, size=shp)
        elif len(shp) == 1:
            p[name] = np.zeros(shp)
        else:
            b = 1.0 / math.sqrt(shp[1])
            p[name] = rng.uniform(-b, b, size=shp)
    return pack(arch, p)


@dataclass
class TrainLog:
    losses: list = field(default_factory=list)
    seconds: float = 0.0
    steps: int = 0


def train(model: Surrogate, X, T, epochs: int, batch: int, lr: float, lr_min: float = 1e-5, seed: int = 0,
          log_every: int = 0, printer=print) -> TrainLog:
    """Adam with a cosine learning-rate schedule over ``epochs`` passes of
    seeded random mini-batches.  ``X``, ``T`` are normalised GPU tensors."""
    import torch
    n = X.shape[0]
    per_epoch = n // batch
    total = epochs * per_epoch
    rng = np.random.default_rng(seed)
    log = TrainLog()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step = 0
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).to(X.device)
        for k in range(per_epoch):
            idx = perm[k * batch:(k + 1) * batch]
            xb = X.index_select(0, idx).contiguous()
            tb = T.index_select(0, idx).contiguous()
            a = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * step / max(total, 1)))
            loss = model.train_step(xb, tb, a)
            log.losses.append(loss)
            step += 1
            if log_every and step % log_every == 0:
                printer(f"step {step}/{total} epoch {ep} loss {np.mean(log.losses[-log_every:]):.5f} lr {a:.2e}")
    torch.cuda.synchronize()
    log.seconds = time.perf_counter() - t0
    log.steps = step
    return log


def predict(model: Surrogate, X, batch: int):
    import torch
    out = []
    for k in range(0, X.shape[0], batch):
        out.append(model.forward(X[k:k + batch].contiguous()))
    return torch.cat(out)


def relative_l2(Y, T):
    """Per-sample ``||Y - T|| / ||T||`` (FP64 sums, by the library), a numpy array."""
    return _relative_l2(Y.contiguous(), T.contiguous())


@dataclass
class TrainedSurrogate:
    """A trained surrogate with its normalisation and its held-out errors."""
    model: Surrogate
    x_scale: float
    t_scale: float
    heldout_error: float          # mean relative L2 over the held-out set
    heldout_max: float = 0.0      # largest held-out relative L2

    def predict(self, f_coarse, batch: int = 32):
        """Coarse averaged strain [B][6][...] (FP32) of coarse forces."""
        import torch
        x = block_mean(f_coarse.contiguous(), 1, scale=1.0 / self.x_scale, dtype=torch.float32)
        y = predict(self.model, x, batch)
        return block_mean(y, 1, scale=self.t_scale)


def averaged_strain(f_fine, tol_rel: float, surrogate: TrainedSurrogate | None, phase, lame, cell: int,
                    kernel=None, prec: str = "f32", max_batch: int = 512):
    """Coarse translation-averaged strain of the forces ``f_fine``
    [B][3][n][n][n], with the source of each field.

    * With the averaged kernel ``kernel`` [6][3][n][n][n] (FP64): the exact
      averaged strain is the kernel convolution; the surrogate's prediction
      of each input is served when its relative L2 error against that is
      within ``tol_rel``, the exact field otherwise (per input).
    * Without it: the surrogate serves every input when its largest held-out
      error is within ``tol_rel``; otherwise every field comes from the
      solver (translated average over every shift of one cell).
    Returns (fields [B][6][n/2]^3 FP32, list of "surrogate" / "kernel" /
    "solver" per input)."""
    import torch
    B = f_fine.shape[0]
    if kernel is not None:
        if f_fine.dtype != kernel.dtype:
            raise TypeError("the forces must have the averaged kernel's dtype")
        exact = restrict2(averaged_strain_from_kernel(kernel, f_fine), dtype=torch.float32)
        if surrogate is None:
            return exact, ["kernel"] * B
        pred = surrogate.predict(restrict2(f_fine))
        err = relative_l2(pred, exact)
        keep = [bool(e <= tol_rel) for e in err]
        idx = torch.tensor([i for i in range(B) if not keep[i]], dtype=torch.long, device=pred.device)
        if idx.numel():
            pred.index_copy_(0, idx, exact.index_select(0, idx))
        return pred, ["surrogate" if k else "kernel" for k in keep]
    if surrogate is not None and surrogate.heldout_max <= tol_rel:
        return surrogate.predict(restrict2(f_fine)), ["surrogate"] * B
    shape = tuple(phase.shape)
    plan = Plan([shape], prec=prec, max_batch=max_batch, refine=(prec == "f32"))
    dt = torch.float64 if prec == "f64" else torch.float32
    out = []
    for b in range(B):
        avg, _ = plan.translate_average(phase, lame, f_fine[b].to(dt).contiguous(), cell_shifts(cell, 3))
        out.append(restrict2(avg[6:12].contiguous(), dtype=torch.float32))
    plan.close()
    return torch.stack(out), ["solver"] * B
