"""Surrogate C ABI checks that need no GPU: exports, parameter layout, and
argument rejection before any HIP call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import fno_oracle as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lsfft_fno.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2601_00822_amd import fno, lsfft
    if not os.path.exists(lsfft.LIB_PATH):
        pytest.fail("liblsfft.so is not built (run __graft_entry__.build())")
    return fno._setup(lsfft.load_library())


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:lsfft_status|int64_t)\s+(lsfft_fno_\w+)\s*\(", text, re.M)))


def test_exports(lib):
    names = declared()
    assert "lsfft_fno_train_step" in names and "lsfft_fno_forward" in names and len(names) == 9
    for name in names:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("kw", [dict(), dict(n=16, modes=4, hidden=64, layers=2), dict(n=8, modes=2, hidden=32, cin=1, cout=2, layers=1)])
def test_param_layout_matches_oracle(lib, kw):
    from paper_2601_00822_amd.fno import FnoArch, param_count, pack, unpack
    a = FnoArch(**kw)
    oa = F.Arch(**{k: getattr(a, k) for k in ("n", "modes", "width", "hidden", "cin", "cout", "layers")})
    assert [(n, s) for n, s in a.layout()] == [(n, s) for n, s in F.param_shapes(oa)]
    total = sum(int(np.prod(s)) * (2 if n.startswith("r") else 1) for n, s in F.param_shapes(oa))
    assert param_count(a) == total
    rng = np.random.default_rng(0)
    p = {n: (rng.normal(size=s) + 1j * rng.normal(size=s)) if n.startswith("r") else rng.normal(size=s)
         for n, s in a.layout()}
    q = unpack(a, pack(a, p))
    for n in p:
        np.testing.assert_allclose(q[n], p[n], rtol=1e-7, atol=1e-7)


@pytest.mark.parametrize("bad", [dict(n=12), dict(n=64), dict(modes=0), dict(modes=17), dict(width=16),
                                 dict(hidden=48), dict(hidden=288), dict(cin=0), dict(cout=33), dict(layers=0),
                                 dict(layers=9)])
def test_bad_arch_rejected(lib, bad):
    from paper_2601_00822_amd.fno import FnoArch, Arch
    a = FnoArch(**bad).c()
    assert lib.lsfft_fno_param_count(C.byref(a)) == 0
    h = C.c_void_p(1)
    assert lib.lsfft_fno_create(C.byref(h), C.byref(a), 4, None) == -1
    assert h.value is None


def test_null_handles(lib):
    from paper_2601_00822_amd.fno import FnoArch
    a = FnoArch().c()
    assert lib.lsfft_fno_create(None, C.byref(a), 4, None) == -1
    h = C.c_void_p()
    assert lib.lsfft_fno_create(C.byref(h), C.byref(a), 0, None) == -1
    assert lib.lsfft_fno_forward(None, 1, None, None) == -1
    assert lib.lsfft_fno_loss_grad(None, 1, None, None, None, None) == -1
    assert lib.lsfft_fno_adam(None, 1e-3, 0.9, 0.999, 1e-8) == -1
    assert lib.lsfft_fno_set_params(None, None) == -1
    assert lib.lsfft_fno_destroy(None) == 0
