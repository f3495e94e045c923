"""GPU checks of the two spectral layouts (rows of nx/2 entries throughout,
or 8-wide kx blocks between the y and outer passes) on the same problems, in
one process through the layout schedule (kind "layout", one per grid):

* FP64 basic scheme: fields bit for bit equal under both layouts, the same
  iteration count, and the oracle's solution (the layout only moves data;
  the per-pencil arithmetic is the same);
* FP64 CG, FP32 with the FP64 defect correction, a warm start and a mixed
  batch of shifted solves: equal to the other layout within rounding (the
  residual sums, taken in another tile order, feed the CG step sizes and the
  correction's stopping test) and to the oracle;
* the kernel convolution (the packed kx = 0 column's partner entries at
  (-ky, -kz) are found through the layout).

Shapes cover the outer tiles narrower than a kx block (FP64, 4 pencils),
y tiles spanning two blocks, ragged y tiles, nx = 16 (one block), 48 and
96 (three and six blocks), and 2D and nx = 24 grids, which have the row
layout only.  Every test prints its case before the first GPU call.
"""
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


def problem(shape, seed, p=0.3):
    rng = np.random.default_rng(seed)
    phase = (rng.random(shape) < p).astype(np.uint8)
    f = gen.bump_force(shape, gen.random_center(shape, seed + 1), 3.0, gen.random_direction(len(shape), seed + 2))
    return phase, f


def solve_both(torch_dev, shape, phase, f, prec="f64", scheme="basic", refine=False, u0=None):
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    dt = torch.float64 if prec == "f64" else torch.float32
    plan = Plan([shape], prec=prec, scheme=scheme, refine=refine)
    assert plan.schedule("layout", 0) == (1 if prec == "f32" else 0, 2)   # FP64 plans start in rows
    res = []
    for lay in (1, 0):
        plan.set_schedule("layout", 0, lay)
        assert plan.schedule("layout", 0)[0] == lay
        kw = {} if u0 is None else dict(u0=torch.from_numpy(u0).to(dev).to(dt))
        out, rep = plan.solve(torch.from_numpy(phase).to(dev), LAME, torch.from_numpy(f).to(dev).to(dt),
                              tol=1e-8, **kw)
        torch.cuda.synchronize()
        res.append(({k: v.double().cpu().numpy() for k, v in out.items()}, rep))
    plan.close()
    return res


# (4, 6, 16): one kx block, y tiles of 6 lines; (6, 12, 48): three blocks;
# (24, 8, 32): 24-point outer pencils; (8, 64, 32): y tiles of 16 kx over two
# blocks; (64, 4, 96): long outer axis, six blocks
SHAPES = [(4, 6, 16), (6, 12, 48), (24, 8, 32), (8, 64, 32), (64, 4, 96)]


@pytest.mark.parametrize("shape", SHAPES)
def test_fp64_basic_bit_for_bit_across_layouts(torch_dev, shape):
    say(f"FP64 basic, blocked vs row layout, {shape}")
    phase, f = problem(shape, 11 + sum(shape))
    (a, ra), (b, rb) = solve_both(torch_dev, shape, phase, f)
    print(f"iters {ra.iters}/{rb.iters} residual {ra.residual:.3e}/{rb.residual:.3e}")
    assert ra.status == 0 and rb.status == 0 and ra.iters == rb.iters
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    assert abs(ra.residual - rb.residual) <= 1e-12 * rb.residual
    ref = O.solve_basic(phase, LAME, f, tol=1e-8)
    assert ref.iters == ra.iters
    assert O.relative_strain_error_voigt(a["eps"], O.to_voigt(ref.eps)) < 1e-10


@pytest.mark.parametrize("shape", [(6, 12, 48), (64, 4, 96)])
def test_fp64_cg_across_layouts(torch_dev, shape):
    say(f"FP64 CG, blocked vs row layout, {shape}")
    phase, f = problem(shape, 31)
    (a, ra), (b, rb) = solve_both(torch_dev, shape, phase, f, scheme="cg")
    print(f"iters {ra.iters}/{rb.iters}")
    assert ra.status == 0 and rb.status == 0 and abs(ra.iters - rb.iters) <= 1
    assert O.relative_strain_error_voigt(a["eps"], b["eps"]) < 1e-10
    ref = O.solve_pcg_displacement(phase, LAME, f, tol=1e-8)
    assert O.relative_strain_error_voigt(a["eps"], O.to_voigt(ref.eps)) < 1e-9


@pytest.mark.parametrize("shape", [(8, 64, 32), (64, 4, 96)])
def test_fp32_refined_across_layouts(torch_dev, shape):
    say(f"FP32 + FP64 correction, blocked vs row layout, {shape}")
    phase, f = problem(shape, 41)
    f = f.astype(np.float32).astype(np.float64)
    (a, ra), (b, rb) = solve_both(torch_dev, shape, phase, f, prec="f32", refine=True)
    print(f"iters {ra.iters}/{rb.iters} residual {ra.residual:.2e}/{rb.residual:.2e}")
    assert ra.status == 0 and rb.status == 0
    assert ra.residual <= 1e-8 and rb.residual <= 1e-8
    ref = O.solve_basic(phase, LAME, f, tol=1e-9)
    for r in (a, b):
        assert O.relative_strain_error_voigt(r["eps"], O.to_voigt(ref.eps)) < 1e-5
    assert O.relative_strain_error_voigt(a["eps"], b["eps"]) < 1e-5


def test_warm_start_across_layouts(torch_dev):
    shape = (6, 12, 48)
    say(f"FP64 warm start, blocked vs row layout, {shape}")
    phase, f = problem(shape, 51)
    u0 = 0.1 * np.random.default_rng(52).normal(size=(3,) + shape)
    (a, ra), (b, rb) = solve_both(torch_dev, shape, phase, f, u0=u0)
    print(f"iters {ra.iters}/{rb.iters}")
    assert ra.iters == rb.iters
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_shifted_batch_across_layouts(torch_dev):
    """Translated averaging of a 3D cell (shared force spectrum, shifted
    phase maps) on both layouts: averages bit for bit equal."""
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    shape = (8, 8, 16)
    say(f"FP64 translated average, 8 shifts, blocked vs row layout, {shape}")
    phase, f = problem(shape, 61)
    shifts = np.asarray([[0, 0, 0], [1, 2, 3], [3, 1, 5], [7, 7, 15], [2, 0, 1], [5, 3, 2], [0, 6, 9], [4, 4, 8]])
    plan = Plan([shape], prec="f64", max_batch=8)
    outs = []
    for lay in (1, 0):
        plan.set_schedule("layout", 0, lay)
        avg, reps = plan.translate_average(torch.from_numpy(phase).to(dev), LAME, torch.from_numpy(f).to(dev),
                                           shifts, tol=1e-8)
        torch.cuda.synchronize()
        outs.append((avg.cpu().numpy(), [r.iters for r in reps]))
    plan.close()
    assert outs[0][1] == outs[1][1]
    np.testing.assert_array_equal(outs[0][0], outs[1][0])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_kernel_convolve_across_layouts(torch_dev, prec):
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    shape = (6, 12, 32)
    say(f"kernel convolution {prec}, blocked vs row layout, {shape}")
    rng = np.random.default_rng(71)
    K = rng.normal(size=(6, 3) + shape)
    F = rng.normal(size=(2, 3) + shape)
    dt = torch.float64 if prec == "f64" else torch.float32
    plan = Plan([shape], prec=prec)
    outs = []
    for lay in (1, 0):
        plan.set_schedule("layout", 0, lay)
        outs.append(plan.kernel_convolve(torch.from_numpy(K).to(dev).to(dt),
                                         torch.from_numpy(F).to(dev).to(dt)).double().cpu().numpy())
    plan.close()
    np.testing.assert_array_equal(outs[0], outs[1])
    Kr = K.astype(np.float32).astype(np.float64) if prec == "f32" else K
    Fr = F.astype(np.float32).astype(np.float64) if prec == "f32" else F
    for b in range(2):
        want = O.kernel_convolve(Kr, Fr[b])
        err = np.abs(outs[0][b] - want).max() / np.abs(want).max()
        assert err < (1e-12 if prec == "f64" else 1e-5), err


def test_layout_schedule_arguments(torch_dev):
    from paper_2601_00822_amd import Plan, LsfftError
    say("layout schedule argument checks")
    plan = Plan([(4, 6, 16), (4, 6, 24), (16, 16)], prec="f32")
    assert plan.schedule("layout", 0) == (1, 2)
    assert plan.schedule("layout", 1) == (0, 1)          # nx = 24: rows only
    assert plan.schedule("layout", 2, dim=2) == (0, 1)   # 2D: rows only
    plan.set_schedule("layout", 0, 0)
    assert plan.schedule("layout", 0) == (0, 2)
    plan.set_schedule("layout", 1, 0)
    for bad in ((1, 1), (0, 2), (3, 0), (-1, 0)):
        with pytest.raises(LsfftError):
            plan.set_schedule("layout", bad[0], bad[1])
    with pytest.raises(LsfftError):
        plan.schedule("layout", 2)                         # grid 2 is 2D
    plan.close()


def test_mixed_layouts_in_one_batch(torch_dev):
    """One batch whose grids use different layouts in the same launches (the
    kernels read the layout per solve): every solve equals its oracle solve
    and, bit for bit, the same batch with the layouts swapped."""
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    shapes = [(8, 8, 32), (6, 12, 48), (4, 6, 24)]
    say(f"FP64 batch over {shapes} with mixed layouts")
    probs, refs = [], []
    for g, shp in enumerate(shapes):
        phase, f = problem(shp, 81 + g)
        probs.append(dict(grid=g, phase=torch.from_numpy(phase).to(dev), lame=LAME, f=torch.from_numpy(f).to(dev)))
        refs.append(O.solve_basic(phase, LAME, f, tol=1e-8))
    plan = Plan(shapes, prec="f64", max_batch=len(shapes))
    assert plan.schedule("layout", 2) == (0, 1)            # nx = 24: rows only
    results = []
    for lays in ((1, 0), (0, 1)):
        plan.set_schedule("layout", 0, lays[0])
        plan.set_schedule("layout", 1, lays[1])
        outs, reps, st = plan.solve_batch(probs, tol=1e-8)
        torch.cuda.synchronize()
        assert st == 0
        results.append(([{k: v.cpu().numpy() for k, v in o.items()} for o in outs], [r.iters for r in reps]))
        for o, r, ref in zip(outs, reps, refs):
            assert r.iters == ref.iters
            assert O.relative_strain_error_voigt(o["eps"].cpu().numpy(), O.to_voigt(ref.eps)) < 1e-10
    plan.close()
    assert results[0][1] == results[1][1]
    for a, b in zip(results[0][0], results[1][0]):
        for k in a:
            np.testing.assert_array_equal(a[k], b[k], err_msg=k)
