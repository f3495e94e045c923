"""ctypes binding of liblsfft (argument marshalling only).

Every step of the solver runs in the HIP kernels of ``liblsfft.so``; this
module checks tensor shapes, dtypes and devices, converts array-order shapes
and shifts to the library's (x, y, z) order, passes raw device pointers and
the current HIP stream, and turns status codes into exceptions.  Torch is
used for device memory and streams only.  There is no fallback: if the
library is missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblsfft.so")

OK, W_STAGNATED = 0, 1
E_ARG, E_ALLOC, E_DEVICE, E_NOCONV, E_NONEQUIL, E_DIVERGED = -1, -2, -3, -4, -5, -6
F32, F64 = 0, 1
BASIC, CG, CG_PLAIN, ANDERSON = 0, 1, 2, 3
SCHEMES = {"basic": BASIC, "cg": CG, "cg_plain": CG_PLAIN, "anderson": ANDERSON}
STRICT_EQUIL, TIMING, REFINE64 = 0x1, 0x2, 0x4
K_XPASS, K_YPASS, K_GREEN, K_REDUCE, K_CGUPD, K_OTHER = range(6)

EXPORTS = [
    "lsfft_plan", "lsfft_solve_bfcs", "lsfft_translate_average", "lsfft_translate_average_batch",
    "lsfft_realization_average", "lsfft_rve_identify", "lsfft_rve_identify_noalloc",
    "lsfft_plan_destroy", "lsfft_status_string", "lsfft_lame_from_young", "lsfft_kernel_times",
    "lsfft_kernel_times_reset", "lsfft_iteration_bytes", "lsfft_schedule_get", "lsfft_schedule_set",
    "lsfft_autotune", "lsfft_tune_cache_lookup", "lsfft_anderson_memory", "lsfft_kernel_convolve",
    "lsfft_block_mean", "lsfft_sample_norms", "lsfft_bump_forces", "lsfft_nonlocal_normal_equations",
    "lsfft_nonlocal_apply", "lsfft_nonlocal_fit",
]
# schedule kinds: the three passes (keyed by transform length) and the
# spectral layout (keyed by the grid's index in the plan)
PASS_KINDS = {"x": 0, "y": 1, "outer": 2, "layout": 3}


class Rve(C.Structure):
    _fields_ = [("radius", C.c_double), ("box_radius", C.c_double), ("fits", C.c_int), ("nbins", C.c_int),
                ("max_eps", C.c_double), ("max_sig", C.c_double)]


class TuneEntry(C.Structure):
    _fields_ = [("kind", C.c_int), ("len", C.c_int), ("variant", C.c_int), ("chosen", C.c_int), ("us", C.c_double)]


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int64 * 3), ("h", C.c_double * 3)]


class Phases(C.Structure):
    _fields_ = [("nphase", C.c_int), ("lame", C.POINTER(C.c_double))]


class Ref(C.Structure):
    _fields_ = [("lambda0", C.c_double), ("mu0", C.c_double)]


class Report(C.Structure):
    _fields_ = [("iters", C.c_int), ("residual", C.c_double), ("removed_mean", C.c_double * 3),
                ("status", C.c_int), ("seconds", C.c_double)]


class AvgGroup(C.Structure):
    _fields_ = [("grid_idx", C.c_int), ("phase", C.c_void_p), ("tab", C.POINTER(Phases)),
                ("c0", C.POINTER(Ref)), ("f", C.c_void_p), ("shifts", C.POINTER(C.c_int32)),
                ("nshift", C.c_int), ("incl_phase", C.c_int), ("avg", C.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblsfft.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "or python paper_2601_00822_amd/build_lib.py")
    lib = C.CDLL(path)
    vp, ip, dp = C.c_void_p, C.c_int, C.c_double
    lib.lsfft_plan.argtypes = [C.POINTER(vp), C.POINTER(Grid), ip, ip, ip, ip, C.c_uint, vp]
    lib.lsfft_plan.restype = ip
    lib.lsfft_solve_bfcs.argtypes = [vp, ip, C.POINTER(ip), C.POINTER(vp), C.POINTER(Phases), C.POINTER(Ref),
                                     C.POINTER(vp), dp, ip, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                     C.POINTER(vp), C.POINTER(Report)]
    lib.lsfft_solve_bfcs.restype = ip
    lib.lsfft_translate_average.argtypes = [vp, ip, vp, C.POINTER(Phases), C.POINTER(Ref), vp,
                                            C.POINTER(C.c_int32), ip, ip, dp, ip, vp, C.POINTER(Report)]
    lib.lsfft_translate_average.restype = ip
    lib.lsfft_translate_average_batch.argtypes = [vp, ip, C.POINTER(AvgGroup), dp, ip, C.POINTER(Report)]
    lib.lsfft_translate_average_batch.restype = ip
    lib.lsfft_realization_average.argtypes = [vp, ip, ip, C.POINTER(vp), C.POINTER(Phases), C.POINTER(Ref), vp,
                                              ip, dp, ip, vp, C.POINTER(Report)]
    lib.lsfft_realization_average.restype = ip
    lib.lsfft_rve_identify.argtypes = [vp, ip, vp, C.POINTER(dp), dp, dp, dp, C.POINTER(dp), ip, C.POINTER(Rve)]
    lib.lsfft_rve_identify.restype = ip
    lib.lsfft_rve_identify_noalloc.argtypes = lib.lsfft_rve_identify.argtypes
    lib.lsfft_rve_identify_noalloc.restype = ip
    lib.lsfft_plan_destroy.argtypes = [vp]
    lib.lsfft_plan_destroy.restype = ip
    lib.lsfft_status_string.argtypes = [ip]
    lib.lsfft_status_string.restype = C.c_char_p
    lib.lsfft_lame_from_young.argtypes = [ip, C.POINTER(dp), C.POINTER(dp)]
    lib.lsfft_lame_from_young.restype = ip
    lib.lsfft_kernel_times.argtypes = [vp, ip, C.POINTER(dp), C.POINTER(C.c_int64)]
    lib.lsfft_kernel_times.restype = ip
    lib.lsfft_kernel_times_reset.argtypes = [vp]
    lib.lsfft_kernel_times_reset.restype = ip
    lib.lsfft_iteration_bytes.argtypes = [vp, ip, ip, C.POINTER(dp)]
    lib.lsfft_iteration_bytes.restype = ip
    lib.lsfft_schedule_get.argtypes = [vp, ip, ip, ip, C.POINTER(ip), C.POINTER(ip)]
    lib.lsfft_schedule_get.restype = ip
    lib.lsfft_schedule_set.argtypes = [vp, ip, ip, ip, ip]
    lib.lsfft_schedule_set.restype = ip
    lib.lsfft_autotune.argtypes = [vp, ip, C.c_char_p, C.POINTER(TuneEntry), ip, C.POINTER(ip)]
    lib.lsfft_autotune.restype = ip
    lib.lsfft_tune_cache_lookup.argtypes = [C.c_char_p, ip, ip, ip, ip]
    lib.lsfft_tune_cache_lookup.restype = ip
    lib.lsfft_anderson_memory.argtypes = [vp, ip]
    lib.lsfft_anderson_memory.restype = ip
    lib.lsfft_kernel_convolve.argtypes = [vp, ip, vp, ip, C.POINTER(vp), C.POINTER(vp)]
    lib.lsfft_kernel_convolve.restype = ip
    lib.lsfft_block_mean.argtypes = [ip, ip, ip, C.POINTER(C.c_int64), ip, dp, vp, vp, vp]
    lib.lsfft_block_mean.restype = ip
    lib.lsfft_sample_norms.argtypes = [ip, ip, C.c_int64, vp, vp, C.POINTER(dp), C.POINTER(dp), vp]
    lib.lsfft_sample_norms.restype = ip
    lib.lsfft_bump_forces.argtypes = [ip, ip, C.POINTER(C.c_int64), ip, C.POINTER(ip), C.POINTER(dp),
                                      C.POINTER(vp), vp]
    lib.lsfft_bump_forces.restype = ip
    lib.lsfft_nonlocal_normal_equations.argtypes = [ip, ip, C.POINTER(C.c_int64), ip, vp, vp, ip, ip, dp,
                                                    C.POINTER(dp), C.POINTER(dp), C.POINTER(dp), vp]
    lib.lsfft_nonlocal_normal_equations.restype = ip
    lib.lsfft_nonlocal_apply.argtypes = [ip, ip, C.POINTER(C.c_int64), ip, vp, ip, ip, C.POINTER(dp), dp, vp, vp]
    lib.lsfft_nonlocal_apply.restype = ip
    lib.lsfft_nonlocal_fit.argtypes = [ip, C.POINTER(dp), C.POINTER(dp), dp, ip, dp, C.POINTER(dp)]
    lib.lsfft_nonlocal_fit.restype = ip
    _lib = lib
    return lib


def _prec_of(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"FP32 or FP64 tensors only, got {t.dtype}")


def _dev_check(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous GPU tensor")


def block_mean(a, factor: int = 2, scale: float = 1.0, dtype=None, spatial: int = 3):
    """Block means over the last ``spatial`` axes of ``a`` (FP32 or FP64 GPU
    tensor), times ``scale``, as ``dtype`` (default: the input's); computed
    by the library (factor 1: a scaled copy)."""
    torch = _torch()
    _dev_check(a, "a")
    nd = spatial
    sp = tuple(a.shape[-nd:])
    nfield = int(np.prod(a.shape[:-nd])) if a.dim() > nd else 1
    n = (C.c_int64 * 3)(*(list(reversed(sp)) + [1] * (3 - nd)))
    dtype = dtype or a.dtype
    out = torch.empty(tuple(a.shape[:-nd]) + tuple(v // factor for v in sp), dtype=dtype, device=a.device)
    st = load_library().lsfft_block_mean(_prec_of(a), _prec_of(out), nfield, n, int(factor), float(scale),
                                         C.c_void_p(a.data_ptr()), C.c_void_p(out.data_ptr()),
                                         C.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st != OK:
        raise LsfftError(st, "lsfft_block_mean")
    return out


def sample_norms(t, y=None):
    """Per-sample norms over all but the first axis: (||y - t|| or ||t||,
    ||t||) as FP64 numpy arrays; computed by the library."""
    torch = _torch()
    _dev_check(t, "t")
    if y is not None:
        _dev_check(y, "y")
        if y.shape != t.shape or y.dtype != t.dtype:
            raise ValueError("y and t must match")
    ns = int(t.shape[0])
    ln = int(t.numel() // ns)
    nd = np.zeros(ns)
    nt = np.zeros(ns)
    st = load_library().lsfft_sample_norms(_prec_of(t), ns, ln, None if y is None else C.c_void_p(y.data_ptr()),
                                           C.c_void_p(t.data_ptr()), nd.ctypes.data_as(C.POINTER(C.c_double)),
                                           nt.ctypes.data_as(C.POINTER(C.c_double)),
                                           C.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st != OK:
        raise LsfftError(st, "lsfft_sample_norms")
    return nd, nt


def relative_l2(y, t):
    """Per-sample ||y - t|| / ||t|| (FP64 numpy), computed by the library."""
    nd, nt = sample_norms(t, y)
    return nd / nt


def bump_forces(shape, params, dtype=None, device=None):
    """Forces ``[len(params)][d][...shape]`` made of smooth bumps, evaluated
    by the library: ``params[i]`` lists (centre in array order, radius,
    direction x first) of force i's bumps."""
    torch = _torch()
    dtype = dtype or torch.float64
    device = device or torch.device("cuda:0")
    d = len(shape)
    out = torch.empty((len(params), d) + tuple(shape), dtype=dtype, device=device)
    nb = (C.c_int * len(params))(*[len(b) for b in params])
    flat = []
    for bumps in params:
        for c, r, v in bumps:
            flat += [float(x) for x in reversed(list(c))] + [float(r)] + [float(x) for x in v]
    arr = np.ascontiguousarray(np.asarray(flat if flat else [0.0], dtype=np.float64))
    ptrs = (C.c_void_p * len(params))(*[out[i].data_ptr() for i in range(len(params))])
    n = (C.c_int64 * 3)(*(list(reversed(shape)) + [1] * (3 - d)))
    st = load_library().lsfft_bump_forces(F64 if dtype == torch.float64 else F32, d, n, len(params), nb,
                                          arr.ctypes.data_as(C.POINTER(C.c_double)), ptrs,
                                          C.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st != OK:
        raise LsfftError(st, "lsfft_bump_forces")
    return out


def _nl_fields(u, name):
    """(prec, d, n[3], nsample) of fields ``[nsample][d][...grid]``."""
    _dev_check(u, name)
    d = u.dim() - 2
    if d not in (2, 3) or u.shape[1] != d:
        raise ValueError(f"{name} must be [nsample][d][...grid] with d = 2 or 3")
    n = (C.c_int64 * 3)(*(list(reversed(tuple(u.shape[2:]))) + [1] * (3 - d)))
    return _prec_of(u), d, n, int(u.shape[0])


def nonlocal_normal_equations(u, gamma, degree: int, delta: float, form: int = 0):
    """(G, g, Gamma . Gamma) of the least-squares fit of the nonlocal
    operator with degree-``degree`` Bernstein kernels of horizon ``delta``
    (``form`` 0: scalar kernel, 1: K1 I + K2 e e^T) to the pairs
    (u_k, Gamma_k), ``[nsample][d][...grid]`` GPU tensors; FP64 numpy,
    computed by the library."""
    torch = _torch()
    prec, d, n, ns = _nl_fields(u, "u")
    _dev_check(gamma, "gamma")
    if gamma.shape != u.shape or gamma.dtype != u.dtype:
        raise ValueError("u and gamma must match")
    nf = (2 if form == 1 else 1) * (degree + 1)
    G = np.zeros((nf, nf))
    g = np.zeros(nf)
    gg = C.c_double(0.0)
    dp = C.POINTER(C.c_double)
    st = load_library().lsfft_nonlocal_normal_equations(prec, d, n, ns, C.c_void_p(u.data_ptr()),
                                                        C.c_void_p(gamma.data_ptr()), int(degree), int(form),
                                                        float(delta), G.ctypes.data_as(dp), g.ctypes.data_as(dp),
                                                        C.byref(gg),
                                                        C.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st != OK:
        raise LsfftError(st, "lsfft_nonlocal_normal_equations")
    return G, g, gg.value


def nonlocal_apply(u, c, delta: float, form: int = 0):
    """L_c[u] of fields ``[nsample][d][...grid]`` (GPU tensor), by the
    library; ``c`` holds (form + 1)(degree + 1) coefficients."""
    torch = _torch()
    prec, d, n, ns = _nl_fields(u, "u")
    c = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
    if form not in (0, 1) or len(c) % (form + 1):
        raise ValueError("form 0 or 1 with (form + 1)(degree + 1) coefficients")
    out = torch.empty_like(u)
    st = load_library().lsfft_nonlocal_apply(prec, d, n, ns, C.c_void_p(u.data_ptr()), len(c) // (form + 1) - 1,
                                             int(form), c.ctypes.data_as(C.POINTER(C.c_double)), float(delta),
                                             C.c_void_p(out.data_ptr()),
                                             C.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st != OK:
        raise LsfftError(st, "lsfft_nonlocal_apply")
    return out


def nonlocal_fit(G, g, lam: float, adam_steps: int = 0, lr: float = 1e-3):
    """Bernstein coefficients from the normal equations: the closed form
    (adam_steps = 0) or Adam from zero; host arithmetic in the library."""
    G = np.ascontiguousarray(np.asarray(G, dtype=np.float64))
    g = np.ascontiguousarray(np.asarray(g, dtype=np.float64))
    nf = len(g)
    if G.shape != (nf, nf):
        raise ValueError("G must be square with the size of g")
    c = np.zeros(nf)
    dp = C.POINTER(C.c_double)
    st = load_library().lsfft_nonlocal_fit(nf, G.ctypes.data_as(dp), g.ctypes.data_as(dp), float(lam),
                                           int(adam_steps), float(lr), c.ctypes.data_as(dp))
    if st != OK:
        raise LsfftError(st, "lsfft_nonlocal_fit")
    return c


class LsfftError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = load_library().lsfft_status_string(status).decode()
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


def status_string(status: int) -> str:
    return load_library().lsfft_status_string(status).decode()


def lame_from_young(table) -> np.ndarray:
    """``[nphase][2]`` (E, nu) to (lambda, mu), computed by the library."""
    t = np.ascontiguousarray(np.asarray(table, dtype=np.float64))
    out = np.zeros_like(t)
    st = load_library().lsfft_lame_from_young(
        t.shape[0], t.ctypes.data_as(C.POINTER(C.c_double)), out.ctypes.data_as(C.POINTER(C.c_double)))
    if st != OK:
        raise LsfftError(st, "lame_from_young")
    return out


@dataclass
class SolveReport:
    iters: int
    residual: float
    removed_mean: tuple
    status: int
    seconds: float


def _report(r: Report, d: int) -> SolveReport:
    return SolveReport(r.iters, r.residual, tuple(r.removed_mean[:d]), r.status, r.seconds)


def _torch():
    import torch
    return torch


class Plan:
    """A solver plan for one or more grids (array-order shapes)."""

    def __init__(self, shapes, prec: str = "f64", scheme: str = "basic", max_batch: int = 1,
                 strict_equil: bool = False, timing: bool = False, spacing=None, refine: bool = False,
                 anderson_memory: int = None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("liblsfft needs a HIP GPU; none is visible")
        self.lib = load_library()
        if isinstance(shapes[0], int):
            shapes = [shapes]
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.prec = prec
        self.dtype = torch.float64 if prec == "f64" else torch.float32
        grids = (Grid * len(self.shapes))()
        for g, shp in enumerate(self.shapes):
            d = len(shp)
            if d not in (2, 3):
                raise ValueError("grids are 2D or 3D")
            grids[g].dim = d
            rev = list(reversed(shp)) + [1] * (3 - d)
            for a in range(3):
                grids[g].n[a] = rev[a]
                grids[g].h[a] = 1.0 if spacing is None else float(list(reversed(spacing[g]))[a] if a < d else 1.0)
        flags = (STRICT_EQUIL if strict_equil else 0) | (TIMING if timing else 0) | (REFINE64 if refine else 0)
        self.stream = torch.cuda.current_stream()
        h = C.c_void_p()
        st = self.lib.lsfft_plan(C.byref(h), grids, len(self.shapes), int(max_batch),
                                 F64 if prec == "f64" else F32, SCHEMES[scheme],
                                 flags, C.c_void_p(self.stream.cuda_stream))
        if st != OK:
            raise LsfftError(st, "lsfft_plan")
        self.handle = h
        if anderson_memory is not None:
            st = self.lib.lsfft_anderson_memory(self.handle, int(anderson_memory))
            if st != OK:
                raise LsfftError(st, "lsfft_anderson_memory")

    # ------------------------------------------------------------------ utils
    def close(self):
        if getattr(self, "handle", None):
            self.lib.lsfft_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, t, shape, dtype, name):
        torch = _torch()
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name} must be a GPU tensor")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return C.c_void_p(t.data_ptr())

    @staticmethod
    def _phases(lame):
        arr = np.ascontiguousarray(np.asarray(lame, dtype=np.float64).reshape(-1, 2))
        ph = Phases(arr.shape[0], arr.ctypes.data_as(C.POINTER(C.c_double)))
        return ph, arr

    @staticmethod
    def _ref(c0):
        if c0 is None:
            return Ref(float("nan"), float("nan"))
        return Ref(float(c0[0]), float(c0[1]))

    # ------------------------------------------------------------------ solves
    def solve_batch(self, problems, tol=1e-8, max_iter=10000, outputs=("eps", "sig", "u")):
        """``problems``: list of dicts with keys grid (index), phase (uint8 GPU
        tensor), lame ([nphase][2]), f ([d][...] GPU tensor), optional c0 and
        optional u0 (starting displacement ``[d][...]`` GPU tensor: given for
        every problem or for none).
        Returns (list of {eps, sig, u} tensors, list of SolveReport, status)."""
        torch = _torch()
        n = len(problems)
        gidx = (C.c_int * n)()
        ph_p = (C.c_void_p * n)()
        f_p = (C.c_void_p * n)()
        tabs = (Phases * n)()
        refs = (Ref * n)()
        eps_p = (C.c_void_p * n)()
        sig_p = (C.c_void_p * n)()
        u_p = (C.c_void_p * n)()
        warm = [pb.get("u0") is not None for pb in problems]
        if any(warm) and not all(warm):
            raise ValueError("u0 must be given for every problem or for none")
        u0_p = (C.c_void_p * n)() if all(warm) else None
        keep = []
        outs = []
        for i, pb in enumerate(problems):
            g = int(pb.get("grid", 0))
            shp = self.shapes[g]
            d = len(shp)
            s = 6 if d == 3 else 3
            gidx[i] = g
            ph_p[i] = self._check(pb["phase"], shp, torch.uint8, "phase")
            f_p[i] = self._check(pb["f"], (d,) + shp, self.dtype, "f")
            if u0_p is not None:
                u0_p[i] = self._check(pb["u0"], (d,) + shp, self.dtype, "u0")
            tabs[i], arr = self._phases(pb["lame"])
            keep.append(arr)
            refs[i] = self._ref(pb.get("c0"))
            o = {}
            dev = pb["f"].device
            if "eps" in outputs:
                o["eps"] = torch.empty((s,) + shp, dtype=self.dtype, device=dev)
                eps_p[i] = o["eps"].data_ptr()
            if "sig" in outputs:
                o["sig"] = torch.empty((s,) + shp, dtype=self.dtype, device=dev)
                sig_p[i] = o["sig"].data_ptr()
            if "u" in outputs:
                o["u"] = torch.empty((d,) + shp, dtype=self.dtype, device=dev)
                u_p[i] = o["u"].data_ptr()
            outs.append(o)
        reps = (Report * n)()
        st = self.lib.lsfft_solve_bfcs(self.handle, n, gidx, ph_p, tabs, refs, f_p, float(tol), int(max_iter),
                                       eps_p, sig_p, u_p, u0_p, reps)
        if st not in (OK, W_STAGNATED, E_NOCONV, E_DIVERGED):
            raise LsfftError(st, "lsfft_solve_bfcs")
        return outs, [_report(reps[i], len(self.shapes[gidx[i]])) for i in range(n)], st

    def solve(self, phase, lame, f, tol=1e-8, max_iter=10000, c0=None, grid=0,
              outputs=("eps", "sig", "u"), u0=None):
        """One solve (optionally warm-started from the displacement ``u0``);
        returns ({eps, sig, u}, SolveReport)."""
        outs, reps, _ = self.solve_batch([dict(grid=grid, phase=phase, lame=lame, f=f, c0=c0, u0=u0)],
                                         tol=tol, max_iter=max_iter, outputs=outputs)
        return outs[0], reps[0]

    # ------------------------------------------------------------------ averaging
    def translate_average_batch(self, groups, tol=1e-8, max_iter=10000):
        """``groups``: list of dicts with keys grid, phase, lame, f, shifts
        (array order ``[n][d]``), optional incl_phase (default 1) and c0.
        Returns (list of FP64 averages ``[2d + 4s + 1][...]``, reports, status)."""
        torch = _torch()
        ng = len(groups)
        arr = (AvgGroup * ng)()
        keep = []
        avgs = []
        total = 0
        for k, gr in enumerate(groups):
            g = int(gr.get("grid", 0))
            shp = self.shapes[g]
            d = len(shp)
            s = 6 if d == 3 else 3
            tab, lame_arr = self._phases(gr["lame"])
            ref = self._ref(gr.get("c0"))
            sh = np.ascontiguousarray(np.asarray(gr["shifts"], dtype=np.int32).reshape(-1, d)[:, ::-1])
            avg = torch.empty((2 * d + 4 * s + 1,) + shp, dtype=torch.float64, device=gr["f"].device)
            keep += [tab, lame_arr, ref, sh]
            arr[k].grid_idx = g
            arr[k].phase = self._check(gr["phase"], shp, torch.uint8, "phase")
            arr[k].tab = C.pointer(tab)
            arr[k].c0 = C.pointer(ref)
            arr[k].f = self._check(gr["f"], (d,) + shp, self.dtype, "f")
            arr[k].shifts = sh.ctypes.data_as(C.POINTER(C.c_int32))
            arr[k].nshift = sh.shape[0]
            arr[k].incl_phase = int(gr.get("incl_phase", 1))
            arr[k].avg = avg.data_ptr()
            avgs.append(avg)
            total += sh.shape[0]
        reps = (Report * total)()
        st = self.lib.lsfft_translate_average_batch(self.handle, ng, arr, float(tol), int(max_iter), reps)
        if st not in (OK, W_STAGNATED, E_NOCONV, E_DIVERGED):
            raise LsfftError(st, "lsfft_translate_average_batch")
        out_reps = []
        k = 0
        for gr in groups:
            d = len(self.shapes[int(gr.get("grid", 0))])
            for _ in range(np.asarray(gr["shifts"]).reshape(-1, d).shape[0]):
                out_reps.append(_report(reps[k], d))
                k += 1
        return avgs, out_reps, st

    def translate_average(self, phase, lame, f, shifts, incl_phase=1, tol=1e-8, max_iter=10000,
                          c0=None, grid=0):
        avgs, reps, st = self.translate_average_batch(
            [dict(grid=grid, phase=phase, lame=lame, f=f, shifts=shifts, incl_phase=incl_phase, c0=c0)],
            tol=tol, max_iter=max_iter)
        return avgs[0], reps

    def realization_average(self, phases, lame, f, incl_phase=1, tol=1e-8, max_iter=10000, c0=None, grid=0):
        """Deterministic-structure average (Eq. 3.8) over the realisations
        ``phases`` (list of uint8 maps of one grid) with the force fixed.
        Returns (FP64 average ``[2d + 4s + 1][...]``, per-realisation reports)."""
        torch = _torch()
        shp = self.shapes[grid]
        d = len(shp)
        s = 6 if d == 3 else 3
        tab, lame_arr = self._phases(lame)
        ref = self._ref(c0)
        n = len(phases)
        ptrs = (C.c_void_p * n)(*[self._check(ph, shp, torch.uint8, "phase") for ph in phases])
        fp = self._check(f, (d,) + shp, self.dtype, "f")
        avg = torch.empty((2 * d + 4 * s + 1,) + shp, dtype=torch.float64, device=f.device)
        reps = (Report * n)()
        st = self.lib.lsfft_realization_average(self.handle, int(grid), n, ptrs, C.byref(tab), C.byref(ref), fp,
                                                int(incl_phase), float(tol), int(max_iter), avg.data_ptr(), reps)
        if st not in (OK, W_STAGNATED, E_NOCONV, E_DIVERGED):
            raise LsfftError(st, "lsfft_realization_average")
        return avg, [_report(reps[k], d) for k in range(n)]

    def rve_identify(self, avg, center, support_radius, tol=1e-3, dr=1.0, grid=0, noalloc=False):
        """RVE of Definition 2.2 from averaged fields ``avg`` (the layout of
        ``translate_average``): ``center`` of the force support in array
        order, voxel units.  Returns a dict with the RVE radius, the cell's
        inscribed radius, whether the RVE plus half the support fits, and the
        radial maxima of |eps| and |sigma| per bin of width ``dr``.  With
        ``noalloc`` the library's allocation-free entry point runs instead."""
        torch = _torch()
        shp = self.shapes[grid]
        d = len(shp)
        s = 6 if d == 3 else 3
        a = self._check(avg, (2 * d + 4 * s + 1,) + shp, torch.float64, "avg")
        c = (C.c_double * 3)(*([float(v) for v in reversed(list(center))] + [0.0] * (3 - d)))
        nmax = 1024
        prof = np.zeros(2 * nmax)
        out = Rve()
        fn = self.lib.lsfft_rve_identify_noalloc if noalloc else self.lib.lsfft_rve_identify
        st = fn(self.handle, int(grid), a, c, float(support_radius), float(tol), float(dr),
                prof.ctypes.data_as(C.POINTER(C.c_double)), nmax, C.byref(out))
        if st != OK:
            raise LsfftError(st, "lsfft_rve_identify")
        nb = out.nbins
        return dict(radius=out.radius, box_radius=out.box_radius, fits=bool(out.fits), nbins=nb,
                    max_eps=out.max_eps, max_sig=out.max_sig, profile_eps=prof[:nb].copy(),
                    profile_sig=prof[nmax:nmax + nb].copy())

    # ------------------------------------------------------------------ kernel convolution
    def kernel_convolve(self, kernel, forces, grid=0):
        """Periodic convolution of ``forces`` [B][d][...] with ``kernel``
        [s][d][...] (the averaged point-force response), through the plan's
        transforms; returns [B][s][...] in the plan precision."""
        torch = _torch()
        shp = self.shapes[grid]
        d = len(shp)
        s = 6 if d == 3 else 3
        kp = self._check(kernel, (s, d) + shp, self.dtype, "kernel")
        B = int(forces.shape[0])
        out = torch.empty((B, s) + shp, dtype=self.dtype, device=forces.device)
        fp = (C.c_void_p * B)(*[self._check(forces[i], (d,) + shp, self.dtype, "force") for i in range(B)])
        op = (C.c_void_p * B)(*[out[i].data_ptr() for i in range(B)])
        st = self.lib.lsfft_kernel_convolve(self.handle, int(grid), kp, B, fp, op)
        if st != OK:
            raise LsfftError(st, "lsfft_kernel_convolve")
        return out

    # ------------------------------------------------------------------ schedules
    def schedule(self, kind: str, length: int, dim: int = 3):
        """(variant in use, number of variants) of pass ``kind`` ("x", "y" or
        "outer") on an axis of ``length`` points; for ``kind`` "layout", of
        the spectral layout of grid ``length`` (its index in the plan): 0
        rows, 1 kx-blocked (3D grids with nx a multiple of 16)."""
        v, n = C.c_int(), C.c_int()
        st = self.lib.lsfft_schedule_get(self.handle, int(dim), PASS_KINDS[kind], int(length), C.byref(v), C.byref(n))
        if st != OK:
            raise LsfftError(st, "lsfft_schedule_get")
        return v.value, n.value

    def set_schedule(self, kind: str, length: int, variant: int, dim: int = 3):
        st = self.lib.lsfft_schedule_set(self.handle, int(dim), PASS_KINDS[kind], int(length), int(variant))
        if st != OK:
            raise LsfftError(st, "lsfft_schedule_set")

    def autotune(self, iters: int = 20, cache_path=None):
        """Time every schedule variant of the plan's 3D grids under each of
        their spectral layouts, keep the faster layout per grid and the
        fastest variants under it; returns the timings as a list of dicts
        (layout entries: kind "layout", len = the grid's index, us = kernel
        time of the three passes per iteration on their fastest variants)."""
        cap = 512
        out = (TuneEntry * cap)()
        n = C.c_int()
        st = self.lib.lsfft_autotune(self.handle, int(iters), None if cache_path is None else str(cache_path).encode(),
                                     out, cap, C.byref(n))
        if st != OK:
            raise LsfftError(st, "lsfft_autotune")
        kinds = {v: k for k, v in PASS_KINDS.items()}
        return [dict(kind=kinds[out[i].kind], len=out[i].len, variant=out[i].variant, chosen=bool(out[i].chosen),
                     us=out[i].us) for i in range(min(n.value, cap))]

    # ------------------------------------------------------------------ timing
    def kernel_times(self, kclass: int):
        ms = C.c_double()
        n = C.c_int64()
        st = self.lib.lsfft_kernel_times(self.handle, kclass, C.byref(ms), C.byref(n))
        if st != OK:
            raise LsfftError(st, "lsfft_kernel_times")
        return ms.value, n.value

    def kernel_times_reset(self):
        self.lib.lsfft_kernel_times_reset(self.handle)

    def iteration_bytes(self, kclass: int, grid: int = 0) -> float:
        b = C.c_double()
        st = self.lib.lsfft_iteration_bytes(self.handle, grid, kclass, C.byref(b))
        if st != OK:
            raise LsfftError(st, "lsfft_iteration_bytes")
        return b.value
