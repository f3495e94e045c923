"""C-ABI checks that need no GPU: the library loads, exports every entry
point the header declares, and rejects bad arguments before any HIP call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import lsfft_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lsfft.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2601_00822_amd import lsfft
    if not os.path.exists(lsfft.LIB_PATH):
        pytest.fail("liblsfft.so is not built (run __graft_entry__.build())")
    return lsfft.load_library()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:lsfft_status|const char\*|int)\s+(lsfft_\w+)\s*\(", text, re.M)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("lsfft_plan", "lsfft_solve_bfcs", "lsfft_translate_average", "lsfft_plan_destroy",
                     "lsfft_status_string"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
    from paper_2601_00822_amd import lsfft
    assert set(lsfft.EXPORTS) == set(declared_functions())


def test_status_strings(lib):
    for s in (0, 1, -1, -2, -3, -4, -5, -6):
        assert lib.lsfft_status_string(s)
    assert b"unknown" in lib.lsfft_status_string(99)


def test_lame_from_young_matches_oracle(lib):
    from paper_2601_00822_amd import lame_from_young, LsfftError
    tab = np.array([[1.0, 0.3], [10.0, 0.3], [0.5, 0.1], [3.0, -0.2]])
    np.testing.assert_allclose(lame_from_young(tab), O.lame_from_young(tab), rtol=1e-15)
    with pytest.raises(LsfftError):
        lame_from_young([[1.0, 0.5]])
    with pytest.raises(LsfftError):
        lame_from_young([[-1.0, 0.3]])


def _grid(dim, n, h=(1.0, 1.0, 1.0)):
    from paper_2601_00822_amd.lsfft import Grid
    g = Grid()
    g.dim = dim
    for a in range(3):
        g.n[a] = n[a]
        g.h[a] = h[a]
    return g


@pytest.mark.parametrize("dim,n,h", [
    (4, (8, 8, 8), (1, 1, 1)),          # dim
    (2, (7, 8, 1), (1, 1, 1)),          # odd length
    (3, (10, 8, 8), (1, 1, 1)),         # prime factor 5
    (3, (512, 8, 8), (1, 1, 1)),        # longer than supported
    (3, (8, 8, 8), (1, 0, 1)),          # spacing
    (2, (8, 8, 1), (1, float("nan"), 1)),
])
def test_plan_rejects_bad_grids(lib, dim, n, h):
    g = _grid(dim, n, h)
    out = C.c_void_p(1)
    assert lib.lsfft_plan(C.byref(out), C.byref(g), 1, 1, 0, 0, 0, None) == -1
    assert out.value is None


def test_plan_rejects_bad_scalars(lib):
    g = _grid(3, (8, 8, 8))
    out = C.c_void_p()
    assert lib.lsfft_plan(None, C.byref(g), 1, 1, 0, 0, 0, None) == -1
    assert lib.lsfft_plan(C.byref(out), C.byref(g), 0, 1, 0, 0, 0, None) == -1   # ngrid
    assert lib.lsfft_plan(C.byref(out), C.byref(g), 1, 0, 0, 0, 0, None) == -1   # max_batch
    assert lib.lsfft_plan(C.byref(out), C.byref(g), 1, 1, 2, 0, 0, None) == -1   # precision
    assert lib.lsfft_plan(C.byref(out), C.byref(g), 1, 1, 0, 5, 0, None) == -1   # scheme
    assert lib.lsfft_plan(C.byref(out), C.byref(g), 1, 1, 0, 0, 0x80, None) == -1  # flags
    assert lib.lsfft_plan(C.byref(out), C.byref(g), 1, 1, 1, 0, 0x4, None) == -1   # FP64 refinement
    assert lib.lsfft_plan(C.byref(out), C.byref(g), 1, 70000, 0, 0, 0x4, None) == -1  # batch too large


def test_calls_on_null_plan(lib):
    from paper_2601_00822_amd.lsfft import Report
    rep = Report()
    assert lib.lsfft_solve_bfcs(None, 1, None, None, None, None, None, 1e-8, 10,
                                None, None, None, None, C.byref(rep)) == -1
    assert lib.lsfft_translate_average(None, 0, None, None, None, None, None, 1, 1, 1e-8, 10,
                                       None, C.byref(rep)) == -1
    assert lib.lsfft_realization_average(None, 0, 1, None, None, None, None, 1, 1e-8, 10,
                                         None, C.byref(rep)) == -1
    assert lib.lsfft_plan_destroy(None) == 0
    ms = C.c_double()
    assert lib.lsfft_kernel_times(None, 0, C.byref(ms), None) == -1


def test_enlargement_lengths_match_the_library(lib):
    # every length the BFUC enlargement steps through passes the plan's
    # argument checks (on a machine without a GPU the plan then fails with
    # LSFFT_E_DEVICE, never LSFFT_E_ARG); lengths outside the set are refused
    from paper_2601_00822_amd.rve import LENGTHS
    for n in LENGTHS:
        g = _grid(2, (n, n, 1))
        out = C.c_void_p()
        st = lib.lsfft_plan(C.byref(out), C.byref(g), 1, 1, 1, 0, 0, None)
        assert st != -1, n
        if st == 0:
            lib.lsfft_plan_destroy(out)
    for n in (10, 18, 20, 512):
        g = _grid(2, (n, n, 1))
        out = C.c_void_p()
        assert lib.lsfft_plan(C.byref(out), C.byref(g), 1, 1, 1, 0, 0, None) == -1, n


def test_tune_cache_lookup(lib):
    """The schedule cache is a flat JSON object of "prec/dimd/kind/len":
    variant pairs; entries outside a length's variant count, malformed text
    and other keys give -1 (the plan then keeps its default)."""
    text = b'{\n  "f32/3d/outer/256": 2,\n  "f32/3d/x/48": 1, "f32/3d/y/128":0,\n  "f32/3d/y/64": 7,\n' \
           b'  "f64/3d/outer/256": 1, "junk": [1, 2], "f32/2d/outer/256": 1\n}'
    look = lib.lsfft_tune_cache_lookup
    assert look(text, 0, 3, 2, 256) == 2
    assert look(text, 0, 3, 0, 48) == 1
    assert look(text, 0, 3, 1, 128) == 0
    assert look(text, 0, 3, 1, 64) == -1        # no such variant
    assert look(text, 1, 3, 2, 256) == -1       # FP64 has the default only
    assert look(text, 0, 2, 2, 256) == -1       # 2D has the default only
    assert look(text, 0, 3, 2, 128) == -1       # no entry
    assert look(text, 0, 3, 0, 16) == -1        # short lengths have the default only
    assert look(b"not json at all", 0, 3, 2, 256) == -1
    assert look(b'{"f32/3d/outer/256": }', 0, 3, 2, 256) == -1
    assert look(None, 0, 3, 2, 256) == -1
    assert look(text, 0, 3, 3, 256) == -1       # kind out of range
