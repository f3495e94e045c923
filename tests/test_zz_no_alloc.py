"""The allocation-free RVE entry point (lsfft_rve_identify_noalloc) against
the allocating one (lsfft_rve_identify) and the oracle, through the C ABI:
two calls in a row on one plan, the second on a smaller grid with smaller
values, so that bins left over from the first call would show."""
import sys

import numpy as np
import pytest

from oracle import lsfft_oracle as O

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"\n[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_00822_amd import load_library
    load_library()
    return torch, torch.device("cuda:0")


def random_avg(shape, seed, scale):
    d = len(shape)
    s = 6 if d == 3 else 3
    rng = np.random.default_rng(seed)
    return scale * rng.normal(size=(2 * d + 4 * s + 1,) + shape) * np.exp(rng.normal(size=shape))


def test_noalloc_matches_allocating_entry_twice(torch_dev):
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    shapes = [(16, 24, 32), (8, 8, 12)]
    plan = Plan(shapes, prec="f64")
    cases = [(0, (3.5, 11.0, 30.25), 1e3, 0.6), (1, (1.0, 7.5, 0.0), 1.0, 0.9)]
    try:
        for grid, center, scale, dr in cases:
            shape = shapes[grid]
            say(f"rve noalloc vs allocating, grid {shape}, dr {dr}")
            avg = random_avg(shape, 10 + grid, scale)
            a = torch.from_numpy(avg).to(dev)
            got = plan.rve_identify(a, center, 3.0, tol=0.2, dr=dr, grid=grid, noalloc=True)
            ref = plan.rve_identify(a, center, 3.0, tol=0.2, dr=dr, grid=grid)
            assert got["nbins"] == ref["nbins"]
            np.testing.assert_array_equal(got["profile_eps"], ref["profile_eps"])
            np.testing.assert_array_equal(got["profile_sig"], ref["profile_sig"])
            for k in ("radius", "box_radius", "fits", "max_eps", "max_sig"):
                assert got[k] == ref[k], k
            radius, fits, pe, ps = O.rve_radius(avg, center, 3.0, 0.2, dr=dr)
            np.testing.assert_array_equal(got["profile_eps"], pe)
            np.testing.assert_array_equal(got["profile_sig"], ps)
            assert got["radius"] == radius and got["fits"] == fits
    finally:
        plan.close()


def test_noalloc_rejects_more_bins_than_the_scratch_holds(torch_dev):
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan, LsfftError, E_ARG
    say("rve noalloc: too many bins is an argument error")
    shape = (8, 8, 8)
    plan = Plan([shape], prec="f64")
    try:
        a = torch.from_numpy(random_avg(shape, 3, 1.0)).to(dev)
        with pytest.raises(LsfftError) as ei:
            plan.rve_identify(a, (4.0, 4.0, 4.0), 2.0, tol=0.1, dr=0.005, noalloc=True)
        assert ei.value.status == E_ARG
        ok = plan.rve_identify(a, (4.0, 4.0, 4.0), 2.0, tol=0.1, dr=0.5, noalloc=True)
        assert ok["nbins"] == int(np.floor(np.sqrt(3 * 16.0) / 0.5)) + 1
    finally:
        plan.close()
