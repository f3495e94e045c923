"""GPU parity of the deterministic-structure average (Sec. 3, Eq. 3.8):
realisations of the microstructure with the force fixed, against the
oracle.  Every test prints its case before the first GPU call."""
import sys

import numpy as np
import pytest

import gen
from oracle import lsfft_oracle as O

pytestmark = pytest.mark.gpu

LAME = O.lame_from_young(gen.Material.two_phase(1.0, 10.0).table())


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


def _maps(shape, seeds, p=0.35):
    return [(np.random.default_rng(s).random(shape) < p).astype(np.uint8) for s in seeds]


@pytest.mark.parametrize("shape,max_batch", [((32, 32), 2), ((12, 16, 8), 5)])
def test_fp64_against_oracle(torch_dev, shape, max_batch):
    say(f"realisation average FP64 {shape}, max_batch {max_batch}")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    maps = _maps(shape, [21, 22, 23, 24, 25])
    f = np.random.default_rng(26).normal(size=(len(shape),) + shape)
    ref, iters = O.realization_average(maps, LAME, f, tol=1e-10)
    plan = Plan([shape], prec="f64", max_batch=max_batch)
    avg, reps = plan.realization_average([torch.from_numpy(m).to(dev) for m in maps], LAME,
                                         torch.from_numpy(f).to(dev), tol=1e-10)
    a = avg.cpu().numpy()
    assert [r.iters for r in reps] == iters
    np.testing.assert_allclose(a, ref, rtol=0, atol=1e-10 * np.abs(ref).max())
    # occupancy: the count of realisations with the inclusion phase is exact;
    # the division by their number may round differently (one ulp)
    np.testing.assert_array_equal(np.rint(a[-1] * len(maps)), np.rint(ref[-1] * len(maps)))
    np.testing.assert_allclose(a[-1], ref[-1], rtol=0, atol=2.3e-16)
    plan.close()


def test_fp32_refined_3d(torch_dev):
    say("realisation average FP32 + FP64 correction 16x16x32")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    shape = (16, 16, 32)
    maps = _maps(shape, [31, 32, 33])
    f = gen.bump_force(shape, (7.3, 8.1, 15.6), 5.0, gen.random_direction(3, 34))
    ref, _ = O.realization_average(maps, LAME, f, tol=1e-10)
    plan = Plan([shape], prec="f32", max_batch=3, refine=True)
    avg, reps = plan.realization_average([torch.from_numpy(m).to(dev) for m in maps], LAME,
                                         torch.from_numpy(f).to(dev).float(), tol=1e-8)
    a = avg.cpu().numpy()
    print("iters", [r.iters for r in reps], "residuals", [f"{r.residual:.1e}" for r in reps])
    assert all(r.status == 0 for r in reps)
    s = 6
    assert O.relative_strain_error_voigt(a[6:6 + s], ref[6:6 + s]) < 1e-5
    assert O.relative_strain_error_voigt(a[18:18 + s], ref[18:18 + s]) < 1e-5
    np.testing.assert_array_equal(np.rint(a[-1] * len(maps)), np.rint(ref[-1] * len(maps)))
    plan.close()


def test_shifted_copies_match_translated_average(torch_dev):
    say("realisation average of shifted copies vs translated average, FP64 8x16x16")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    shape = (8, 16, 16)
    ph = _maps(shape, [41])[0]
    f = gen.bump_force(shape, (3.5, 7.2, 9.9), 4.0, gen.random_direction(3, 42))
    shifts = np.array([[0, 0, 0], [1, 3, 5], [7, 15, 2]], dtype=np.int32)
    reals = [np.ascontiguousarray(np.roll(ph, shift=tuple(int(c) for c in chi), axis=(0, 1, 2))) for chi in shifts]
    plan = Plan([shape], prec="f64", max_batch=3)
    a, _ = plan.realization_average([torch.from_numpy(r).to(dev) for r in reals], LAME,
                                    torch.from_numpy(f).to(dev), tol=1e-10)
    b, _ = plan.translate_average(torch.from_numpy(ph).to(dev), LAME, torch.from_numpy(f).to(dev), shifts, tol=1e-10)
    torch.testing.assert_close(a, b, rtol=0, atol=1e-12 * float(b.abs().max()))
    plan.close()
