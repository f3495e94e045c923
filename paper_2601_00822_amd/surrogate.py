"""Dataset, training and evaluation of the learned surrogate (Sec. 6, Fig. 5
blocks 2-3) around the HIP solver and the HIP surrogate kernels.

Dataset (the compressed dataset of Eq. 3.7 for one periodic
microstructure): the translation average over every shift of one cell is a
linear map of the force that commutes with grid translations, i.e. a
periodic convolution.  Its kernel, the averaged strain response to a unit
point force at the origin along each axis, comes from three
``translate_average`` calls of the batched solver (3 x cell^3 solves).  The
averaged strain of any force is then that kernel convolved with the force;
the convolution (a Fourier-space product) is data preparation, done with
torch's FFT in FP64.  Forces and targets are restricted to the coarse grid
by block means.

Training and inference run entirely in the surrogate kernels (bf16 MFMA,
fp32 accumulation, Adam); this module only moves batches and schedules the
learning rate.  The solver supplies the held-out targets the surrogate is
measured against, and stays the fallback (``averaged_strain``).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from .fno import FnoArch, Surrogate, pack
from .lsfft import Plan


def cell_shifts(cell: int, d: int = 3) -> np.ndarray:
    """Every integer shift inside one cell, ``[cell^d][d]`` in array order."""
    g = np.stack(np.meshgrid(*([np.arange(cell)] * d), indexing="ij"), axis=-1)
    return g.reshape(-1, d).astype(np.int32)


def averaged_strain_kernel(phase, lame, cell: int, prec: str = "f64", max_batch: int = 512, tol: float = 1e-8):
    """``K[c][j]`` = the translation-averaged strain component ``c`` (Voigt)
    for a unit point force along axis ``j`` (x first) at the origin; FP64
    torch tensor ``[6][3][n][n][n]``.  Returns (K, per-shift reports)."""
    import torch
    shape = tuple(phase.shape)
    d = len(shape)
    if d != 3:
        raise ValueError("the surrogate dataset is 3D")
    plan = Plan([shape], prec=prec, max_batch=max_batch, refine=(prec == "f32"))
    dt = torch.float64 if prec == "f64" else torch.float32
    shifts = cell_shifts(cell, d)
    cols, reps = [], []
    for j in range(d):
        f = torch.zeros((d,) + shape, dtype=dt, device=phase.device)
        f[(j,) + (0,) * d] = 1.0
        avg, r = plan.translate_average(phase, lame, f, shifts, tol=tol)
        cols.append(avg[2 * d:2 * d + 6].clone())
        reps += r
    plan.close()
    return torch.stack(cols, dim=1), reps


def kernel_spectrum(K):
    import torch
    return torch.fft.rfftn(K, dim=(-3, -2, -1))


def averaged_strain_from_kernel(Khat, f):
    """``f`` [B][3][n][n][n] -> averaged strain [B][6][n][n][n] (FP64)."""
    import torch
    fh = torch.fft.rfftn(f.to(torch.float64), dim=(-3, -2, -1))
    eh = torch.einsum("cjzyx,bjzyx->bczyx", Khat, fh)
    return torch.fft.irfftn(eh, s=f.shape[-3:], dim=(-3, -2, -1))


def restrict2(a):
    """2 x 2 x 2 block means of the last three axes."""
    s = a.shape
    n = s[-1]
    return a.reshape(s[:-3] + (n // 2, 2, n // 2, 2, n // 2, 2)).mean(dim=(-5, -3, -1))


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
    """Per-sample ``||Y - T|| / ||T||`` (FP64), a CPU numpy array."""
    import torch
    B = Y.shape[0]
    d = (Y.double() - T.double()).reshape(B, -1)
    return (torch.linalg.norm(d, dim=1) / torch.linalg.norm(T.double().reshape(B, -1), dim=1)).cpu().numpy()


@dataclass
class TrainedSurrogate:
    """A trained surrogate with its normalisation and held-out error; the
    solver is used instead whenever that error exceeds the caller's bound."""
    model: Surrogate
    x_scale: float
    t_scale: float
    heldout_error: float

    def predict(self, f_coarse, batch: int = 32):
        return predict(self.model, (f_coarse / self.x_scale).float().contiguous(), batch) * self.t_scale


def averaged_strain(f_fine, tol_rel: float, surrogate: TrainedSurrogate | None, phase, lame, cell: int,
                    prec: str = "f32", max_batch: int = 512):
    """Coarse translation-averaged strain of the forces ``f_fine``
    [B][3][n][n][n]: from the surrogate when its held-out error is within
    ``tol_rel``, else from the solver (every shift of one cell)."""
    import torch
    if surrogate is not None and surrogate.heldout_error <= tol_rel:
        return surrogate.predict(restrict2(f_fine.double())), "surrogate"
    shape = tuple(phase.shape)
    plan = Plan([shape], prec=prec, max_batch=max_batch, refine=(prec == "f32"))
    dt = torch.float64 if prec == "f64" else torch.float32
    out = []
    for b in range(f_fine.shape[0]):
        avg, _ = plan.translate_average(phase, lame, f_fine[b].to(dt).contiguous(), cell_shifts(cell, 3))
        out.append(restrict2(avg[6:12]))
    plan.close()
    return torch.stack(out), "solver"
