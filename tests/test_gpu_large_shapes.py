"""GPU parity against the FP64 oracle on the kernel specializations that the
large workloads run: transform lengths 48, 64, 96 and 256 on every axis, the
XCD-ordered y pass (256-point y pencils), full 8-pencil outer tiles on
256-point outer pencils, mixed 48/64/96 batches, and the full 256-shift
translated average of the 2D 64x64 workload.

Shapes are array order (nz, ny, nx); the other axes are kept small so the
oracle finishes in seconds.  Bars: FP64 iterate for iterate (same iteration
count, relative strain error <= 1e-10); FP32 <= 1e-5 against the oracle's
FP64 solution at residual 1e-8.  Every test prints its case before the first
GPU call.
"""
import sys

import numpy as np
import pytest

import gen
from oracle import lsfft_oracle as O

pytestmark = pytest.mark.gpu

LAME10 = O.lame_from_young(gen.Material.two_phase(1.0, 10.0).table())


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


def rand_phase(shape, seed, p=0.35):
    return (np.random.default_rng(seed).random(shape) < p).astype(np.uint8)


def gpu_solve(torch_dev, shape, phase, lame, f, prec="f64", scheme="basic", tol=1e-8, max_iter=10000,
              refine=False):
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    dt = torch.float64 if prec == "f64" else torch.float32
    plan = Plan([shape], prec=prec, scheme=scheme, refine=refine)
    out, rep = plan.solve(torch.from_numpy(np.ascontiguousarray(phase)).to(dev), lame,
                          torch.from_numpy(np.ascontiguousarray(f)).to(dev).to(dt),
                          tol=tol, max_iter=max_iter)
    torch.cuda.synchronize()
    res = {k: v.double().cpu().numpy() for k, v in out.items()}
    plan.close()
    return res, rep


def check_iterates(torch_dev, shape, phase, lame, f, js, tol=1e-8, scheme="basic"):
    solver = O.solve_basic if scheme == "basic" else O.solve_pcg_displacement
    for j in js:
        ref = solver(phase, lame, f, tol=tol, max_iter=j)
        res, rep = gpu_solve(torch_dev, shape, phase, lame, f, tol=tol, max_iter=j, scheme=scheme)
        assert rep.iters == ref.iters, (j, rep.iters, ref.iters)
        err = O.relative_strain_error_voigt(res["eps"], O.to_voigt(ref.eps))
        assert err < 1e-10, (j, err)
        assert np.abs(res["u"] - ref.u).max() < 1e-10 * np.abs(ref.u).max()
        assert np.abs(res["sig"] - O.to_voigt(ref.sig)).max() < 1e-10 * np.abs(ref.sig).max()
    ref = solver(phase, lame, f, tol=tol)
    res, rep = gpu_solve(torch_dev, shape, phase, lame, f, tol=tol, scheme=scheme)
    assert rep.status == 0 and ref.status == 0
    assert rep.iters == ref.iters, (rep.iters, ref.iters)
    err = O.relative_strain_error_voigt(res["eps"], O.to_voigt(ref.eps))
    print(f"iters={rep.iters} residual={rep.residual:.3e} err={err:.3e}")
    assert err < 1e-10, err
    return rep, ref


# (4, 256, 16): 256-point y pencils, 8 kx columns per y tile, XCD-ordered
# units; (256, 4, 16): 256-point outer pencils, full 8-pencil tiles (FP32)
# and 4-pencil tiles (FP64); 48/64/96 on the y and outer axes.
LARGE_AXIS_SHAPES = [(4, 256, 16), (256, 4, 16), (48, 96, 8), (96, 48, 8), (64, 64, 8)]


@pytest.mark.parametrize("shape", LARGE_AXIS_SHAPES)
def test_fp64_iterates_large_axes(torch_dev, shape):
    say(f"FP64 iterate parity on long y / outer axes {shape}")
    phase = rand_phase(shape, 71)
    f = gen.bump_force(shape, gen.random_center(shape, 72), 3.0, gen.random_direction(3, 73))
    check_iterates(torch_dev, shape, phase, LAME10, f, js=[0, 1, 3])


@pytest.mark.parametrize("shape", [(4, 256, 16), (256, 4, 16)])
def test_fp64_cg_iterates_256_axes(torch_dev, shape):
    say(f"FP64 CG iterate parity on 256-point axes {shape}")
    phase = rand_phase(shape, 74, 0.3)
    lame = O.lame_from_young(gen.Material.two_phase(1.0, 100.0).table())
    f = gen.bump_force(shape, gen.random_center(shape, 75), 3.0, gen.random_direction(3, 76))
    check_iterates(torch_dev, shape, phase, lame, f, js=[0, 1, 4], scheme="cg")


@pytest.mark.parametrize("shape", [(8, 8, 48), (8, 8, 96), (6, 4, 256)])
def test_fp64_iterates_long_x(torch_dev, shape):
    say(f"FP64 iterate parity on long x rows {shape}")
    phase = rand_phase(shape, 81)
    f = gen.bump_force(shape, gen.random_center(shape, 82), 3.0, gen.random_direction(3, 83))
    check_iterates(torch_dev, shape, phase, LAME10, f, js=[0, 2])


@pytest.mark.parametrize("shape", [(8, 8, 48), (8, 8, 96), (4, 256, 16), (256, 4, 16), (48, 96, 8),
                                   (96, 48, 8)])
@pytest.mark.parametrize("refine", [False, True])
def test_fp32_large_axes_vs_oracle(torch_dev, shape, refine):
    """FP32 transforms on the long axes (x at 48 and 96 through the x pass's
    dense 1536-entry tiles; y and outer at 48, 96 and 256), with and without
    the FP64 defect correction, against the oracle's FP64 solution at 1e-8."""
    say(f"FP32 {'+ FP64 correction ' if refine else ''}vs oracle {shape}")
    phase = rand_phase(shape, 91)
    f = gen.bump_force(shape, gen.random_center(shape, 92), 3.0, gen.random_direction(3, 93))
    f = f.astype(np.float32).astype(np.float64)   # the force the FP32 plan sees
    ref = O.solve_basic(phase, LAME10, f, tol=1e-8)
    res, rep = gpu_solve(torch_dev, shape, phase, LAME10, f, prec="f32", tol=1e-8, refine=refine)
    err = O.relative_strain_error_voigt(res["eps"], O.to_voigt(ref.eps))
    serr = O.relative_strain_error_voigt(res["sig"], O.to_voigt(ref.sig))
    uerr = np.linalg.norm(res["u"] - ref.u) / np.linalg.norm(ref.u)
    print(f"status={rep.status} iters={rep.iters}/{ref.iters} residual={rep.residual:.3e} "
          f"err={err:.3e} serr={serr:.3e} uerr={uerr:.3e}")
    if refine:
        assert rep.status == 0 and rep.residual <= 1e-8
    else:
        assert rep.status in (0, 1)
    assert err < 1e-5 and serr < 1e-5 and uerr < 1e-5


def mixed_problems(seed0):
    """Solves on 48, 64 and 96-point axes in every position, two contrasts."""
    shapes = [(48, 8, 64), (8, 96, 48), (64, 48, 8), (6, 64, 96)]
    probs = []
    for g, shp in enumerate(shapes):
        for k, kappa in enumerate((3.0, 12.0)):
            ph = rand_phase(shp, seed0 + 10 * g + k, 0.3)
            f = gen.bump_force(shp, gen.random_center(shp, seed0 + 50 + 10 * g + k), 4.0,
                               gen.random_direction(3, seed0 + 90 + 10 * g + k))
            probs.append((g, ph, O.lame_from_young(gen.Material.two_phase(1.0, kappa).table()), f))
    return shapes, probs


def test_fp64_mixed_48_64_96_batch(torch_dev):
    """One batch of solves of 48/64/96-point axes (four grids, two contrasts
    each): every solve equals its oracle solve element by element, with the
    same iteration count."""
    say("FP64 mixed 48/64/96 batch vs oracle")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    shapes, probs = mixed_problems(500)
    refs = [O.solve_basic(ph, lame, f, tol=1e-8) for _, ph, lame, f in probs]
    plan = Plan(shapes, prec="f64", max_batch=len(probs))
    pb = [dict(grid=g, phase=torch.from_numpy(ph).to(dev), lame=lame, f=torch.from_numpy(f).to(dev))
          for g, ph, lame, f in probs]
    outs, reps, st = plan.solve_batch(pb, tol=1e-8)
    plan.close()
    assert st == 0
    for o, r, ref in zip(outs, reps, refs):
        assert r.iters == ref.iters, (r.iters, ref.iters)
        e = o["eps"].cpu().numpy()
        assert O.relative_strain_error_voigt(e, O.to_voigt(ref.eps)) < 1e-10
        np.testing.assert_allclose(e, O.to_voigt(ref.eps), rtol=0, atol=1e-10 * np.abs(ref.eps).max())
        np.testing.assert_allclose(o["u"].cpu().numpy(), ref.u, rtol=0, atol=1e-10 * np.abs(ref.u).max())


def test_fp32_refined_mixed_48_64_96_batch(torch_dev):
    """The batched configuration (FP32 transforms, FP64 correction) on mixed
    48/64/96 grids: FP64 residual <= 1e-8 for every solve and strain within
    the FP32 bar of the oracle."""
    say("FP32 + FP64 correction mixed 48/64/96 batch vs oracle")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    shapes, probs = mixed_problems(600)
    probs = [(g, ph, lame, f.astype(np.float32).astype(np.float64)) for g, ph, lame, f in probs]
    refs = [O.solve_basic(ph, lame, f, tol=1e-9) for _, ph, lame, f in probs]
    plan = Plan(shapes, prec="f32", max_batch=len(probs), refine=True)
    pb = [dict(grid=g, phase=torch.from_numpy(ph).to(dev), lame=lame, f=torch.from_numpy(f).to(dev).float())
          for g, ph, lame, f in probs]
    outs, reps, st = plan.solve_batch(pb, tol=1e-8)
    plan.close()
    assert st == 0
    for o, r, ref in zip(outs, reps, refs):
        assert r.residual <= 1e-8
        err = O.relative_strain_error_voigt(o["eps"].double().cpu().numpy(), O.to_voigt(ref.eps))
        assert err < 1e-5, err


def test_2d_64_full_shift_average(torch_dev):
    """The 2D 64x64 workload's translated average over all 256 intra-cell
    shifts (FP64), against the oracle's literal average (microstructure
    shifted, Eqs. 3.3-3.6): same iteration counts, every accumulator
    component element by element."""
    say("2D 64x64 (4x4 cells of 16x16): 256-shift translated average vs oracle")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    shape = (64, 64)
    phase, _ = gen.inclusion_per_cell(shape, 16, 0.2)
    f = gen.bump_force(shape, gen.random_center(shape, 0), 8.0, [1.0, 0.0])
    shifts = gen.all_shifts(16, 2)
    ref, iters = O.translate_average(phase, LAME10, f, shifts, tol=1e-8)
    plan = Plan([shape], prec="f64", max_batch=256)
    avg, reps = plan.translate_average(torch.from_numpy(phase).to(dev), LAME10, torch.from_numpy(f).to(dev),
                                       shifts, tol=1e-8)
    plan.close()
    a = avg.cpu().numpy()
    assert [r.iters for r in reps] == list(iters)
    for k in range(a.shape[0]):
        scale = max(np.abs(ref[k]).max(), 1e-300)
        np.testing.assert_allclose(a[k], ref[k], rtol=0, atol=1e-10 * scale, err_msg=f"component {k}")
    np.testing.assert_array_equal(a[-1], ref[-1])
