"""ctypes binding of the surrogate part of liblsfft (argument marshalling only).

The forward pass, the gradients and the Adam updates all run in the HIP
kernels behind ``include/lsfft_fno.h``; this module checks shapes, packs and
unpacks the flat fp32 parameter vector and passes device pointers.  There is
no fallback: without the library or a GPU the calls raise.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from .lsfft import LsfftError, OK, load_library


class Arch(C.Structure):
    _fields_ = [("n", C.c_int), ("modes", C.c_int), ("width", C.c_int), ("hidden", C.c_int),
                ("cin", C.c_int), ("cout", C.c_int), ("layers", C.c_int)]


@dataclass(frozen=True)
class FnoArch:
    """Architecture of the surrogate (defaults: 32^3 grid, 12 modes, width
    32, 4 layers, projection 32 -> 128 -> 6, 3 input channels)."""
    n: int = 32
    modes: int = 12
    width: int = 32
    hidden: int = 128
    cin: int = 3
    cout: int = 6
    layers: int = 4

    @property
    def nmodes(self) -> int:
        return 4 * self.modes ** 3

    def c(self) -> Arch:
        return Arch(self.n, self.modes, self.width, self.hidden, self.cin, self.cout, self.layers)

    def layout(self):
        """(name, shape) of every parameter in packing order; the spectral
        weights ``r{l}`` are complex ``[modes][width][width]`` packed as
        interleaved (re, im) fp32."""
        out = [("lift_w", (self.width, self.cin)), ("lift_b", (self.width,))]
        for l in range(self.layers):
            out += [(f"w{l}", (self.width, self.width)), (f"b{l}", (self.width,)),
                    (f"r{l}", (self.nmodes, self.width, self.width))]
        out += [("proj1_w", (self.hidden, self.width)), ("proj1_b", (self.hidden,)),
                ("proj2_w", (self.cout, self.hidden)), ("proj2_b", (self.cout,))]
        return out


def pack(arch: FnoArch, params: dict) -> np.ndarray:
    """Flat fp32 vector from a dict of arrays (complex for ``r{l}``)."""
    parts = []
    for name, shp in arch.layout():
        a = np.asarray(params[name])
        if tuple(a.shape) != tuple(shp):
            raise ValueError(f"{name}: shape {a.shape}, expected {shp}")
        if name.startswith("r"):
            a = np.stack([a.real, a.imag], axis=-1)
        parts.append(np.ascontiguousarray(a, dtype=np.float32).ravel())
    return np.concatenate(parts)


def unpack(arch: FnoArch, flat) -> dict:
    """Dict of float64 arrays (complex for ``r{l}``) from a flat vector."""
    flat = np.asarray(flat, dtype=np.float64)
    out, off = {}, 0
    for name, shp in arch.layout():
        k = int(np.prod(shp)) * (2 if name.startswith("r") else 1)
        a = flat[off:off + k]
        off += k
        if name.startswith("r"):
            a = a.reshape(shp + (2,))
            out[name] = a[..., 0] + 1j * a[..., 1]
        else:
            out[name] = a.reshape(shp)
    return out


def _setup(lib):
    if getattr(lib, "_fno_ready", False):
        return lib
    vp, ip = C.c_void_p, C.c_int
    lib.lsfft_fno_param_count.argtypes = [C.POINTER(Arch)]
    lib.lsfft_fno_param_count.restype = C.c_int64
    lib.lsfft_fno_create.argtypes = [C.POINTER(vp), C.POINTER(Arch), ip, vp]
    lib.lsfft_fno_create.restype = ip
    lib.lsfft_fno_set_params.argtypes = [vp, vp]
    lib.lsfft_fno_set_params.restype = ip
    lib.lsfft_fno_get_params.argtypes = [vp, vp]
    lib.lsfft_fno_get_params.restype = ip
    lib.lsfft_fno_forward.argtypes = [vp, ip, vp, vp]
    lib.lsfft_fno_forward.restype = ip
    lib.lsfft_fno_loss_grad.argtypes = [vp, ip, vp, vp, vp, C.POINTER(C.c_double)]
    lib.lsfft_fno_loss_grad.restype = ip
    lib.lsfft_fno_adam.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float]
    lib.lsfft_fno_adam.restype = ip
    lib.lsfft_fno_train_step.argtypes = [vp, ip, vp, vp, C.c_float, C.POINTER(C.c_double)]
    lib.lsfft_fno_train_step.restype = ip
    lib.lsfft_fno_destroy.argtypes = [vp]
    lib.lsfft_fno_destroy.restype = ip
    lib._fno_ready = True
    return lib


def param_count(arch: FnoArch) -> int:
    a = arch.c()
    return int(_setup(load_library()).lsfft_fno_param_count(C.byref(a)))


class Surrogate:
    """A surrogate instance on the current GPU for batches of up to
    ``max_batch`` samples."""

    def __init__(self, arch: FnoArch = FnoArch(), max_batch: int = 32):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the surrogate kernels need a HIP GPU; none is visible")
        self.lib = _setup(load_library())
        self.arch = arch
        self.max_batch = int(max_batch)
        self.nparam = param_count(arch)
        if self.nparam <= 0:
            raise ValueError(f"unsupported architecture {arch}")
        self.stream = torch.cuda.current_stream()
        h = C.c_void_p()
        a = arch.c()
        st = self.lib.lsfft_fno_create(C.byref(h), C.byref(a), self.max_batch, C.c_void_p(self.stream.cuda_stream))
        if st != OK:
            raise LsfftError(st, "lsfft_fno_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.lsfft_fno_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _io(self, t, channels, batch, name):
        import torch
        n = self.arch.n
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float32:
            raise TypeError(f"{name} must be a float32 GPU tensor")
        if tuple(t.shape) != (batch, channels, n, n, n) or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous [{batch}][{channels}][{n}][{n}][{n}]")
        return C.c_void_p(t.data_ptr())

    def set_params(self, flat):
        """Load packed parameters (numpy or GPU tensor of ``nparam`` fp32)."""
        import torch
        t = torch.as_tensor(np.asarray(flat, dtype=np.float32) if not isinstance(flat, torch.Tensor) else flat)
        t = t.to(device="cuda", dtype=torch.float32).contiguous()
        if t.numel() != self.nparam:
            raise ValueError(f"expected {self.nparam} parameters, got {t.numel()}")
        st = self.lib.lsfft_fno_set_params(self.handle, C.c_void_p(t.data_ptr()))
        if st != OK:
            raise LsfftError(st, "lsfft_fno_set_params")

    def get_params(self):
        import torch
        t = torch.empty(self.nparam, dtype=torch.float32, device="cuda")
        st = self.lib.lsfft_fno_get_params(self.handle, C.c_void_p(t.data_ptr()))
        if st != OK:
            raise LsfftError(st, "lsfft_fno_get_params")
        return t

    def forward(self, x, out=None):
        import torch
        b = int(x.shape[0])
        if not 1 <= b <= self.max_batch:
            raise ValueError(f"batch {b} outside [1, {self.max_batch}]")
        px = self._io(x, self.arch.cin, b, "x")
        n = self.arch.n
        y = out if out is not None else torch.empty((b, self.arch.cout, n, n, n), dtype=torch.float32, device="cuda")
        py = self._io(y, self.arch.cout, b, "y")
        st = self.lib.lsfft_fno_forward(self.handle, b, px, py)
        if st != OK:
            raise LsfftError(st, "lsfft_fno_forward")
        return y

    def loss_grad(self, x, t, want_grad=True):
        import torch
        b = int(x.shape[0])
        px, pt = self._io(x, self.arch.cin, b, "x"), self._io(t, self.arch.cout, b, "t")
        g = torch.empty(self.nparam, dtype=torch.float32, device="cuda") if want_grad else None
        loss = C.c_double()
        st = self.lib.lsfft_fno_loss_grad(self.handle, b, px, pt, C.c_void_p(g.data_ptr()) if g is not None else None,
                                          C.byref(loss))
        if st != OK:
            raise LsfftError(st, "lsfft_fno_loss_grad")
        return loss.value, g

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        st = self.lib.lsfft_fno_adam(self.handle, float(lr), float(beta1), float(beta2), float(eps))
        if st != OK:
            raise LsfftError(st, "lsfft_fno_adam")

    def train_step(self, x, t, lr):
        b = int(x.shape[0])
        px, pt = self._io(x, self.arch.cin, b, "x"), self._io(t, self.arch.cout, b, "t")
        loss = C.c_double()
        st = self.lib.lsfft_fno_train_step(self.handle, b, px, pt, float(lr), C.byref(loss))
        if st != OK:
            raise LsfftError(st, "lsfft_fno_train_step")
        return loss.value
