"""Plain float64 NumPy oracle of the learned nonlocal surrogate.

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

The surrogate is a nonlocal neural operator in the sense of Eq. 6.10: every
hidden layer is ``z <- A(W z + b + K z)``, ``A`` the activation, ``W z + b``
the local (pointwise) part and ``K`` an integral operator with a learned
kernel.  Sec. 6 names the Fourier neural operator among the admissible
families but fixes no architecture; the readings used here are:

* ``K`` is a periodic convolution applied in Fourier space and truncated to
  the low modes: on the half spectrum of the (z, y, x) grid of ``n`` points
  per axis (x the real-to-half axis), keep ``kx`` in ``[0, m)`` and signed
  ``ky, kz`` in ``[-m, m)``; there the channel vector is multiplied by a
  learned complex matrix per mode, ``Y[o] = sum_i X[i] R[mode][i][o]``; all
  other modes are dropped.  The transform pair is NumPy's (forward
  unnormalised, inverse with ``1/n^3``), so the real output of ``K`` is
  ``(1/n^3) sum over kept modes of w_kx Re(Y e^{i k.x})`` with ``w = 1`` on
  ``kx = 0`` and 2 elsewhere.
* ``A`` is the exact GELU ``x Phi(x)``, applied after every hidden layer.
* A pointwise lift (input channels -> width) precedes the hidden layers and a
  two-layer pointwise projection (width -> hidden -> output, GELU between)
  follows them.
* Loss: mean over the batch of the relative L2 error ``||y - t|| / ||t||``.
* Optimiser: Adam with bias correction.

Mode index ``m = (iz * 2M + iy) * M + kx`` with ``iy, iz`` in ``[0, 2M)``
standing for the signed wavenumbers ``0..M-1, -M..-1``.

``bf16=True`` rounds every operand of the matrix products (weights,
activations and incoming gradients) to bfloat16 the way a kernel with bf16
operands and wide accumulation sees them (round to float32, then to the
nearest bf16, ties to even); sums stay float64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SQRT2 = math.sqrt(2.0)


# --------------------------------------------------------------------------
# bfloat16 rounding of operands
# --------------------------------------------------------------------------

def round_bf16(a):
    """Round to float32, then to the nearest bfloat16 (ties to even); NaN
    and infinities pass through.  Returns float64 values."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        return round_bf16(a.real) + 1j * round_bf16(a.imag)
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    finite = np.isfinite(f)
    out = np.where(finite, r, u).astype(np.uint32).view(np.float32)
    return out.astype(np.float64)


def _q(a, bf16):
    return round_bf16(a) if bf16 else a


# --------------------------------------------------------------------------
# activation
# --------------------------------------------------------------------------

_erf = np.vectorize(math.erf, otypes=[np.float64])


def gelu(x):
    """Exact GELU ``x Phi(x) = x (1 + erf(x / sqrt 2)) / 2``."""
    return 0.5 * x * (1.0 + _erf(x / SQRT2))


def gelu_grad(x):
    """``d/dx [x Phi(x)] = Phi(x) + x phi(x)``."""
    return 0.5 * (1.0 + _erf(x / SQRT2)) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


# --------------------------------------------------------------------------
# architecture
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class Arch:
    n: int = 32          # grid points per axis
    modes: int = 12      # M
    width: int = 32
    hidden: int = 128
    cin: int = 3
    cout: int = 6
    layers: int = 4

    @property
    def nmodes(self):
        return 4 * self.modes ** 3

    def mode_index(self):
        """(kz, ky, kx) array indices of the kept modes on the rfft grid, in
        mode order."""
        M, n = self.modes, self.n
        signed = list(range(M)) + list(range(n - M, n))
        kz, ky, kx = np.meshgrid(signed, signed, np.arange(M), indexing="ij")
        return kz.ravel(), ky.ravel(), kx.ravel()


def param_shapes(a: Arch):
    """Names and shapes of the parameters, in packing order."""
    out = [("lift_w", (a.width, a.cin)), ("lift_b", (a.width,))]
    for l in range(a.layers):
        out += [(f"w{l}", (a.width, a.width)), (f"b{l}", (a.width,)),
                (f"r{l}", (a.nmodes, a.width, a.width))]
    out += [("proj1_w", (a.hidden, a.width)), ("proj1_b", (a.hidden,)),
            ("proj2_w", (a.cout, a.hidden)), ("proj2_b", (a.cout,))]
    return out


# --------------------------------------------------------------------------
# spectral convolution (the integral operator K of Eq. 6.10)
# --------------------------------------------------------------------------

def spectral_forward(h, r, a: Arch, bf16=False):
    """``h`` [B][C][n][n][n] real, ``r`` [modes][C][C] complex -> (K h, the
    kept input modes [B][C][modes])."""
    kz, ky, kx = a.mode_index()
    H = np.fft.rfftn(h, axes=(2, 3, 4))[:, :, kz, ky, kx]
    Y = np.einsum("bim,mio->bom", _q(H, bf16), _q(r, bf16))
    full = np.zeros(h.shape[:2] + (a.n, a.n, a.n // 2 + 1), dtype=np.complex128)
    full[:, :, kz, ky, kx] = Y
    return np.fft.irfftn(full, s=(a.n, a.n, a.n), axes=(2, 3, 4)), H


def spectral_backward(g, H, r, a: Arch, bf16=False):
    """Given dL/d(K h) = g, return (dL/dh, dL/dr).

    With ``K h = (1/n^3) sum_k w_k Re(Y_k e^{ik.x})`` and the complex
    gradient convention ``dL/dRe + i dL/dIm``: ``dL/dY_k = (w_k/n^3) rfft(g)_k``;
    for ``Y = X R``: ``dL/dX = dL/dY R^H`` and ``dL/dR = X^H dL/dY``; for
    ``X_k = sum_x h(x) e^{-ik.x}``: ``dL/dh = sum_k Re(dL/dX_k e^{ik.x})``."""
    kz, ky, kx = a.mode_index()
    n3 = float(a.n ** 3)
    w = np.where(kx == 0, 1.0, 2.0)
    G = np.fft.rfftn(g, axes=(2, 3, 4))[:, :, kz, ky, kx] * (w / n3)
    Gq = _q(G, bf16)
    dr = np.einsum("bim,bom->mio", np.conj(_q(H, bf16)), Gq)
    dX = np.einsum("bom,mio->bim", Gq, np.conj(_q(r, bf16)))
    # sum_k Re(dX_k e^{ik.x}) over the kept half-spectrum modes, no weights:
    # an inverse real transform of dX * n^3 / w_k
    full = np.zeros(g.shape[:2] + (a.n, a.n, a.n // 2 + 1), dtype=np.complex128)
    full[:, :, kz, ky, kx] = dX * (n3 / w)
    return np.fft.irfftn(full, s=(a.n, a.n, a.n), axes=(2, 3, 4)), dr


def _pw(w, b, h, bf16):
    """Pointwise layer ``w h + b`` over [B][C][...]."""
    y = np.einsum("oi,bi...->bo...", _q(w, bf16), _q(h, bf16))
    if b is not None:
        y = y + b.reshape((1, -1) + (1,) * (h.ndim - 2))
    return y


def forward(params, x, a: Arch, bf16=False, keep=False):
    """Surrogate output [B][cout][n][n][n]; with ``keep`` also the tape."""
    tape = {}
    h = _pw(params["lift_w"], params["lift_b"], x, bf16)
    tape["h0"] = h
    for l in range(a.layers):
        s, H = spectral_forward(h, params[f"r{l}"], a, bf16)
        pre = _pw(params[f"w{l}"], params[f"b{l}"], h, bf16) + s
        tape[f"H{l}"] = H
        tape[f"pre{l}"] = pre
        h = gelu(pre)
        tape[f"h{l + 1}"] = h
    p1 = _pw(params["proj1_w"], params["proj1_b"], h, bf16)
    z = gelu(p1)
    y = _pw(params["proj2_w"], params["proj2_b"], z, bf16)
    tape["p1"], tape["z"] = p1, z
    return (y, tape) if keep else y


def loss_and_grad_y(y, t):
    """Mean relative L2 error over the batch and its gradient in y."""
    B = y.shape[0]
    d = (y - t).reshape(B, -1)
    tn = np.linalg.norm(t.reshape(B, -1), axis=1)
    en = np.linalg.norm(d, axis=1)
    loss = float(np.mean(en / tn))
    g = d / (np.maximum(en, 1e-300) * tn)[:, None] / B
    return loss, g.reshape(y.shape)


def backward(params, x, t, a: Arch, bf16=False):
    """Loss and the gradient of every parameter (dict)."""
    y, tp = forward(params, x, a, bf16, keep=True)
    loss, gy = loss_and_grad_y(y, t)
    grads = {}
    red = (0,) + tuple(range(2, x.ndim))

    def wgrad(g, h):
        B = g.shape[0]
        return np.einsum("bov,biv->oi", _q(g, bf16).reshape(B, g.shape[1], -1), _q(h, bf16).reshape(B, h.shape[1], -1))

    def pw_back(w, h, g, name):
        grads[name + "_w"] = wgrad(g, h)
        grads[name + "_b"] = g.sum(axis=red)
        return np.einsum("oi,bo...->bi...", _q(w, bf16), _q(g, bf16))

    gz = pw_back(params["proj2_w"], tp["z"], gy, "proj2")
    gp1 = gz * gelu_grad(tp["p1"])
    gh = pw_back(params["proj1_w"], tp[f"h{a.layers}"], gp1, "proj1")
    for l in reversed(range(a.layers)):
        gpre = gh * gelu_grad(tp[f"pre{l}"])
        h = tp[f"h{l}"]
        grads[f"w{l}"] = wgrad(gpre, h)
        grads[f"b{l}"] = gpre.sum(axis=red)
        gh_local = np.einsum("oi,bo...->bi...", _q(params[f"w{l}"], bf16), _q(gpre, bf16))
        gh_spec, grads[f"r{l}"] = spectral_backward(gpre, tp[f"H{l}"], params[f"r{l}"], a, bf16)
        gh = gh_local + gh_spec
    pw_back(params["lift_w"], x, gh, "lift")
    return loss, grads


def adam_step(params, grads, state, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), in place; complex parameters are
    treated as pairs of real parameters.  ``step`` counts from 1."""
    for k, g in grads.items():
        m, v = state.setdefault(k, (np.zeros_like(g), np.zeros_like(g)))
        if np.iscomplexobj(g):
            m = beta1 * m + (1 - beta1) * g
            v = beta2 * v + (1 - beta2) * (g.real ** 2 + 1j * g.imag ** 2)
            mh, vh = m / (1 - beta1 ** step), v / (1 - beta2 ** step)
            params[k] = params[k] - lr * (mh.real / (np.sqrt(vh.real) + eps) + 1j * mh.imag / (np.sqrt(vh.imag) + eps))
        else:
            m = beta1 * m + (1 - beta1) * g
            v = beta2 * v + (1 - beta2) * g * g
            mh, vh = m / (1 - beta1 ** step), v / (1 - beta2 ** step)
            params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
        state[k] = (m, v)
