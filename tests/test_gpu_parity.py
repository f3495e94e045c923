"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Every test prints the case it is about to run before the first GPU call.
Bars: FP64 relative strain error <= 1e-10 (iterate for iterate and at
convergence, same iteration counts); FP32 <= 1e-5 against the oracle's FP64
solution at residual 1e-8.
"""
import sys

import numpy as np
import pytest

import gen
from oracle import dense
from oracle import lsfft_oracle as O

pytestmark = pytest.mark.gpu

MAT10 = gen.Material.two_phase(1.0, 10.0)
LAME10 = O.lame_from_young(MAT10.table())


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


def rand_force(shape, seed):
    return np.random.default_rng(seed).normal(size=(len(shape),) + tuple(shape))


def gpu_solve(torch_dev, shape, phase, lame, f, prec="f64", scheme="basic", tol=1e-8, max_iter=10000, c0=None):
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    dt = torch.float64 if prec == "f64" else torch.float32
    plan = Plan([shape], prec=prec, scheme=scheme)
    out, rep = plan.solve(torch.from_numpy(np.ascontiguousarray(phase)).to(dev), lame,
                          torch.from_numpy(np.ascontiguousarray(f)).to(dev).to(dt),
                          tol=tol, max_iter=max_iter, c0=c0)
    torch.cuda.synchronize()
    res = {k: v.double().cpu().numpy() for k, v in out.items()}
    plan.close()
    return res, rep


def inputs_2d_64(seed=0):
    shape = (64, 64)
    phase, _ = gen.inclusion_per_cell(shape, 16, 0.2)
    f = gen.bump_force(shape, gen.random_center(shape, seed), 8.0, [1.0, 0.0])
    return shape, phase, f


# ---------------------------------------------------------------- closed forms on the GPU

@pytest.mark.parametrize("shape,m", [((16, 16), (3, -2)), ((8, 8, 8), (1, 2, -3)), ((12, 16, 24), (2, -1, 5))])
def test_homogeneous_plane_wave(torch_dev, shape, m):
    say(f"plane wave {shape}")
    d = len(shape)
    lame = np.array([[1.1, 0.7]])
    phase = np.zeros(shape, dtype=np.uint8)
    pos = gen.grid_positions(shape)
    xi = np.array([2 * np.pi * m[a] / shape[d - 1 - a] for a in range(d)])
    arg = sum(xi[a] * pos[d - 1 - a] for a in range(d))
    avec = np.array([0.3, -1.0, 0.5][:d])
    f = np.stack([avec[c] * np.cos(arg) for c in range(d)])
    lam, mu = lame[0]
    n = xi / np.linalg.norm(xi)
    k2 = xi @ xi
    N = np.outer(n, n) / ((lam + 2 * mu) * k2) + (np.eye(d) - np.outer(n, n)) / (mu * k2)
    u_exact = np.stack([(N @ avec)[c] * np.cos(arg) for c in range(d)])
    res, rep = gpu_solve(torch_dev, shape, phase, lame, f, tol=1e-12)
    assert rep.iters == 0 and rep.status == 0
    np.testing.assert_allclose(res["u"], u_exact, atol=1e-13)


@pytest.mark.parametrize("shape", [(8, 8), (16, 16), (4, 4, 4), (6, 6, 6)])
def test_dense_direct_solve(torch_dev, shape):
    say(f"dense pin {shape}")
    phase = rand_phase(shape, 1)
    f = rand_force(shape, 2)
    u, e, s = dense.dense_solve(phase, LAME10, f)
    res, rep = gpu_solve(torch_dev, shape, phase, LAME10, f, tol=1e-13)
    assert rep.status == 0
    assert O.relative_strain_error_voigt(res["eps"], O.to_voigt(e)) < 1e-10
    assert np.abs(res["u"] - u).max() < 1e-10 * np.abs(u).max()
    assert np.abs(res["sig"] - O.to_voigt(s)).max() < 1e-10 * np.abs(s).max()


# ---------------------------------------------------------------- iterate for iterate (FP64)

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
        assert abs(rep.residual - ref.residual) <= 1e-8 * ref.residual + 1e-15
    # converged
    ref = solver(phase, lame, f, tol=tol)
    res, rep = gpu_solve(torch_dev, shape, phase, lame, f, tol=tol, scheme=scheme)
    assert rep.status == 0 and ref.status == 0
    assert rep.iters == ref.iters, (rep.iters, ref.iters)
    assert rep.residual <= tol
    err = O.relative_strain_error_voigt(res["eps"], O.to_voigt(ref.eps))
    assert err < 1e-10, err
    np.testing.assert_allclose(rep.removed_mean, ref.removed_mean, atol=1e-14)
    return rep, ref


def test_2d_64_fp64_iterates(torch_dev):
    """64x64 plane strain, one disk per 16x16 cell (vf 0.2, contrast 10),
    bump R = 8 along x, reference medium = mean of extreme Lame constants,
    basic scheme to 1e-8."""
    say("2D 64x64 FP64 iterate parity")
    shape, phase, f = inputs_2d_64(0)
    rep, ref = check_iterates(torch_dev, shape, phase, LAME10, f, js=[0, 1, 2, 7, 30])
    print(f"iters={rep.iters} residual={rep.residual:.3e}")


@pytest.mark.parametrize("shape", [(16, 16, 16), (8, 12, 16), (12, 24, 48), (6, 24, 96), (8, 4, 32)])
def test_3d_fp64_iterates(torch_dev, shape):
    say(f"3D FP64 iterate parity {shape}")
    phase = rand_phase(shape, 5)
    f = gen.bump_force(shape, gen.random_center(shape, 3), 4.0, gen.random_direction(3, 4))
    check_iterates(torch_dev, shape, phase, LAME10, f, js=[0, 1, 4])


@pytest.mark.parametrize("shape", [(32, 48), (96, 24), (4, 256), (256, 8)])
def test_2d_fp64_shapes(torch_dev, shape):
    say(f"2D FP64 shapes {shape}")
    phase = rand_phase(shape, 7)
    f = rand_force(shape, 8)
    check_iterates(torch_dev, shape, phase, LAME10, f, js=[1, 3])


def plane_force(shape, seed, nyquist_only=False):
    """Force with content in the x planes kx = 0 and kx = nx/2 only, each with
    its own random (y, z) profile: f = a(y, z) + (-1)^x b(y, z)."""
    rng = np.random.default_rng(seed)
    d = len(shape)
    rest = shape[:-1]
    nx = shape[-1]
    sign = (-1.0) ** np.arange(nx)
    a = rng.normal(size=(d,) + rest + (1,))
    b = rng.normal(size=(d,) + rest + (1,))
    f = b * sign
    if not nyquist_only:
        f = f + a
    return np.broadcast_to(f, (d,) + tuple(shape)).copy()


@pytest.mark.parametrize("shape,nyq", [((8, 12, 16), False), ((6, 8, 32), True), ((24, 32), False), ((12, 16), True)])
def test_fp64_x_zero_and_nyquist_planes(torch_dev, shape, nyq):
    """The x planes kx = 0 and kx = nx/2 share one packed column on the GPU;
    a force living on those planes only (or on the Nyquist plane alone) is
    solved iterate for iterate like the oracle, which keeps the planes apart."""
    say(f"FP64 force on the kx = 0 / nx/2 planes {shape} nyquist_only={nyq}")
    phase = rand_phase(shape, 21)
    f = plane_force(shape, 22, nyq)
    check_iterates(torch_dev, shape, phase, LAME10, f, js=[0, 1, 3])


@pytest.mark.parametrize("shape", [(4, 8, 128), (8, 64), (4, 8, 256)])
def test_fp32_staged_x_zero_and_nyquist_planes(torch_dev, shape):
    """The staged FP32 x pass unpacks the kx = 0 / nx/2 entry by value (no
    address select): a force on those planes converges to the oracle's
    solution within the FP32 bar."""
    say(f"FP32 staged x tiles, force on the kx = 0 / nx/2 planes {shape}")
    phase = rand_phase(shape, 23)
    f = plane_force(shape, 24)
    ref = O.solve_basic(phase, LAME10, f, tol=1e-8)
    res, rep = gpu_solve(torch_dev, shape, phase, LAME10, f, prec="f32", tol=1e-6)
    err = O.relative_strain_error_voigt(res["eps"], O.to_voigt(ref.eps))
    print(f"iters={rep.iters} residual={rep.residual:.3e} err={err:.3e}")
    assert rep.status in (0, 1)
    assert err < 1e-5


def test_cg_iterates(torch_dev):
    say("CG 2D 32x32 and 3D 12x16x16 FP64")
    for shape in [(32, 32), (12, 16, 16)]:
        phase = rand_phase(shape, 11, 0.3)
        lame = O.lame_from_young(gen.Material.two_phase(1.0, 50.0).table())
        f = rand_force(shape, 12)
        rep, ref = check_iterates(torch_dev, shape, phase, lame, f, js=[0, 1, 3, 6], tol=1e-9, scheme="cg")
        basic = O.solve_basic(phase, lame, f, tol=1e-9)
        assert rep.iters < basic.iters


def test_explicit_reference_medium(torch_dev):
    say("explicit C0")
    shape = (16, 16)
    phase = rand_phase(shape, 21)
    f = rand_force(shape, 22)
    lam0, mu0 = O.reference_medium(LAME10)
    ref = O.solve_basic(phase, LAME10, f, lam0=1.3 * lam0, mu0=1.3 * mu0, tol=1e-10)
    res, rep = gpu_solve(torch_dev, shape, phase, LAME10, f, tol=1e-10, c0=(1.3 * lam0, 1.3 * mu0))
    assert rep.iters == ref.iters
    assert O.relative_strain_error_voigt(res["eps"], O.to_voigt(ref.eps)) < 1e-10


# ---------------------------------------------------------------- FP32

def test_fp32_3d_vs_fp64_oracle(torch_dev):
    """FP32 transforms and updates, FP64 residual: relative strain error
    against the oracle's FP64 solution at 1e-8 stays <= 1e-5."""
    say("FP32 3D 32^3 vs FP64 oracle")
    shape = (32, 32, 32)
    phase, _ = gen.inclusion_per_cell(shape, 16, 0.25)
    f = gen.bump_force(shape, gen.random_center(shape, 1), 12.0, gen.random_direction(3, 2))
    ref = O.solve_basic(phase, LAME10, f, tol=1e-8)
    res, rep = gpu_solve(torch_dev, shape, phase, LAME10, f, prec="f32", tol=1e-8)
    err = O.relative_strain_error_voigt(res["eps"], O.to_voigt(ref.eps))
    print(f"fp32: status={rep.status} iters={rep.iters} residual={rep.residual:.3e} err={err:.3e}")
    assert rep.status in (0, 1)
    assert err < 1e-5


def test_fp32_2d_64(torch_dev):
    say("FP32 2D 64x64")
    shape, phase, f = inputs_2d_64(1)
    ref = O.solve_basic(phase, LAME10, f, tol=1e-8)
    res, rep = gpu_solve(torch_dev, shape, phase, LAME10, f, prec="f32", tol=1e-8)
    err = O.relative_strain_error_voigt(res["eps"], O.to_voigt(ref.eps))
    print(f"fp32 2D: status={rep.status} iters={rep.iters} residual={rep.residual:.3e} err={err:.3e}")
    assert rep.status in (0, 1)
    assert err < 1e-5


@pytest.mark.parametrize("shape", [(4, 6, 128), (6, 12, 128), (6, 16, 64), (4, 6, 256), (24, 128), (48, 64),
                                   (4, 6, 96), (8, 12, 96), (6, 16, 48), (4, 12, 48), (24, 96), (96, 48)])
def test_fp32_staged_x_tiles(torch_dev, shape):
    """FP32 x pass with row tiles staged by direct global->LDS loads (nx = 64,
    128, 256: 2048-entry tiles of 64, 32 or 16 rows; nx = 48,
    96: dense 1536-entry tiles of 64 and 32 rows): single, several and ragged
    row tiles, 2D and 3D."""
    say(f"FP32 staged x tiles {shape}")
    phase = rand_phase(shape, 51)
    f = rand_force(shape, 52)
    ref = O.solve_basic(phase, LAME10, f, tol=1e-8)
    res, rep = gpu_solve(torch_dev, shape, phase, LAME10, f, prec="f32", tol=1e-8)
    err = O.relative_strain_error_voigt(res["eps"], O.to_voigt(ref.eps))
    serr = O.relative_strain_error_voigt(res["sig"], O.to_voigt(ref.sig))
    print(f"status={rep.status} iters={rep.iters}/{ref.iters} residual={rep.residual:.3e} err={err:.3e} serr={serr:.3e}")
    assert rep.status in (0, 1)
    assert err < 1e-5 and serr < 1e-5


@pytest.mark.parametrize("shape", [(256, 16), (256, 8, 8), (256, 4, 12)])
def test_fp32_outer_axis_256(torch_dev, shape):
    """FP32 outer pass on 256-point pencils: 8 kx columns per tile (fewer
    when nx / 2 is smaller), ragged y lines."""
    say(f"FP32 outer axis 256 {shape}")
    phase = rand_phase(shape, 61)
    f = rand_force(shape, 62)
    ref = O.solve_basic(phase, LAME10, f, tol=1e-8)
    res, rep = gpu_solve(torch_dev, shape, phase, LAME10, f, prec="f32", tol=1e-8)
    err = O.relative_strain_error_voigt(res["eps"], O.to_voigt(ref.eps))
    print(f"status={rep.status} iters={rep.iters}/{ref.iters} residual={rep.residual:.3e} err={err:.3e}")
    assert rep.status in (0, 1)
    assert err < 1e-5


def test_fp32_staged_x_tiles_shifted(torch_dev):
    """Shifted microstructures in the staged x pass: x shifts that are and are
    not multiples of 16 (vector and byte reads of the phase map)."""
    say("FP32 staged x tiles, translated average 4x8x128")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    shape = (4, 8, 128)
    phase = rand_phase(shape, 53)
    f = gen.bump_force(shape, (1.7, 3.2, 40.5), 3.0, gen.random_direction(3, 54))
    shifts = np.array([[0, 0, 0], [1, 2, 16], [3, 1, 5], [2, 5, 37]], dtype=np.int32)
    ref, _ = O.translate_average(phase, LAME10, f, shifts, tol=1e-10)
    plan = Plan([shape], prec="f32", max_batch=4)
    avg, reps = plan.translate_average(torch.from_numpy(phase).to(dev), LAME10,
                                       torch.from_numpy(f).to(dev).float(), shifts, tol=1e-8)
    a = avg.cpu().numpy()
    print("iters", [r.iters for r in reps])
    s = 6
    assert O.relative_strain_error_voigt(a[6:6 + s], ref[6:6 + s]) < 1e-5
    np.testing.assert_array_equal(a[-1], ref[-1])
    plan.close()


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("nx", [48, 96])
def test_fp32_staged_x_tiles_1536_shifted(torch_dev, nx, variant):
    """Shifted microstructures in the dense x tiles of nx = 48 and 96 (1536
    entries in schedule variant 0, 768 in variant 1): x shifts that are
    multiples of 12 (word or half-word reads of the phase map) and others
    (byte reads), against the oracle's translated average."""
    say(f"FP32 staged dense x tiles (variant {variant}), translated average 4x6x{nx}")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    shape = (4, 6, nx)
    phase = rand_phase(shape, 57)
    f = gen.bump_force(shape, (1.7, 2.2, nx / 2 + 0.5), 3.0, gen.random_direction(3, 58))
    shifts = np.array([[0, 0, 0], [1, 2, 12], [3, 1, 5], [2, 5, nx - 12]], dtype=np.int32)   # 4: exact averages
    ref, _ = O.translate_average(phase, LAME10, f, shifts, tol=1e-10)
    plan = Plan([shape], prec="f32", max_batch=len(shifts))
    plan.set_schedule("x", nx, variant)
    avg, reps = plan.translate_average(torch.from_numpy(phase).to(dev), LAME10,
                                       torch.from_numpy(f).to(dev).float(), shifts, tol=1e-8)
    a = avg.cpu().numpy()
    print("iters", [r.iters for r in reps])
    s = 6
    assert O.relative_strain_error_voigt(a[6:6 + s], ref[6:6 + s]) < 1e-5
    np.testing.assert_array_equal(a[-1], ref[-1])
    plan.close()


# ---------------------------------------------------------------- batches

def test_batch_mixed_grids(torch_dev):
    """One batch holding solves of different sizes and dimensions; each equals
    its own oracle solve."""
    say("batch mixed grids")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    shapes = [(16, 16, 16), (24, 24, 24), (32, 32), (8, 16, 12)]
    plan = Plan(shapes, prec="f64", max_batch=8)
    probs, refs = [], []
    for g, shp in enumerate(shapes):
        for k in range(2):
            ph = rand_phase(shp, 100 + 10 * g + k)
            f = rand_force(shp, 200 + 10 * g + k)
            c = 2.0 + 10 * k + g
            lame = O.lame_from_young(gen.Material.two_phase(1.0, c).table())
            probs.append(dict(grid=g, phase=torch.from_numpy(ph).to(dev), lame=lame, f=torch.from_numpy(f).to(dev)))
            refs.append(O.solve_basic(ph, lame, f, tol=1e-9))
    outs, reps, st = plan.solve_batch(probs, tol=1e-9)
    for o, r, ref in zip(outs, reps, refs):
        assert r.iters == ref.iters
        assert O.relative_strain_error_voigt(o["eps"].cpu().numpy(), O.to_voigt(ref.eps)) < 1e-10
    # more solves than max_batch: processed in successive batches
    plan2 = Plan(shapes, prec="f64", max_batch=3)
    outs2, reps2, _ = plan2.solve_batch(probs, tol=1e-9)
    for o, o2 in zip(outs, outs2):
        assert torch.equal(o["eps"], o2["eps"])
    plan.close()
    plan2.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_mixed_dims_rule_in_y_pass(torch_dev, prec):
    """Batch of 3D and 2D solves with different iteration counts: inside
    a captured round the stopping rule runs in the next y pass (the 2D solves
    have no y tiles), in a timed plan it runs in its own kernel.  Both give
    the same iterates bit for bit, and every solve stopped at residual 1e-6
    is within 1e-4 of its converged oracle solution."""
    say(f"{prec} batch 3D + 2D, stopping rule in the y pass vs on its own")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    shapes = [(16, 16, 16), (32, 32), (8, 16, 12), (24, 24)]
    probs, refs = [], []
    for g, shp in enumerate(shapes):
        for k in range(2):
            ph = rand_phase(shp, 300 + 10 * g + k)
            f = rand_force(shp, 400 + 10 * g + k)
            lame = O.lame_from_young(gen.Material.two_phase(1.0, 2.0 + 20 * k + 3 * g).table())
            ft = torch.from_numpy(f).to(dev)
            probs.append(dict(grid=g, phase=torch.from_numpy(ph).to(dev), lame=lame,
                              f=ft if prec == "f64" else ft.float()))
            refs.append(O.solve_basic(ph, lame, f, tol=1e-9))
    res = []
    for timing in (False, True):
        plan = Plan(shapes, prec=prec, max_batch=8, timing=timing)
        outs, reps, _ = plan.solve_batch(probs, tol=1e-6)
        torch.cuda.synchronize()
        res.append(([o["eps"].cpu() for o in outs], [r.iters for r in reps]))
        plan.close()
    assert len(set(res[0][1])) > 1          # the solves stop at different iterations
    assert res[0][1] == res[1][1]
    for a, b in zip(res[0][0], res[1][0]):
        assert torch.equal(a, b)
    # residual 1e-6 against the converged oracle solution, contrast <= 31
    for e, ref in zip(res[0][0], refs):
        assert O.relative_strain_error_voigt(e.double().numpy(), O.to_voigt(ref.eps)) < 1e-4


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_many_solves_stopping_together(torch_dev, prec):
    """256 shifted solves of a point force, most of them stopping within a few
    iterations of each other inside one captured round: the stopping rule in
    the y pass must leave every running solve intact (each workgroup takes one
    gate decision per unit).  Captured and timed plans agree bit for bit."""
    say(f"{prec}: 256 solves stopping together, captured vs timed plan")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    n, cell = 32, 8
    phase = torch.from_numpy(gen.tile_cell(gen.rsa_cell(cell, 3, 0.2, 1.5, 2.5, seed=4)[0], (n, n, n))).to(dev)
    dt = torch.float64 if prec == "f64" else torch.float32
    tol = 1e-10 if prec == "f64" else 1e-4
    f = torch.zeros((3, n, n, n), dtype=dt, device=dev)
    f[0, 0, 0, 0] = 1.0
    shifts = gen.sample_shifts(cell, 3, 256, 5)
    res = []
    for timing in (False, True):
        plan = Plan([(n, n, n)], prec=prec, max_batch=256, timing=timing)
        avg, reps = plan.translate_average(phase, LAME10, f, shifts, tol=tol)
        torch.cuda.synchronize()
        res.append((avg.cpu(), [(r.status, r.iters) for r in reps]))
        plan.close()
    assert all(st == 0 for st, _ in res[0][1]), [x for x in res[0][1] if x[0] != 0][:5]
    assert res[0][1] == res[1][1]
    assert torch.equal(res[0][0], res[1][0])


# ---------------------------------------------------------------- translated averaging

@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_translate_average_2d(torch_dev, prec):
    say(f"translated average 2D {prec}")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    shape = (32, 32)
    phase = gen.tile_cell(gen.inclusion_per_cell((8, 8), 8, 0.25)[0], shape).copy()
    phase[0, 1] = 1
    f = gen.bump_force(shape, (13.2, 17.9), 6.0, [0.8, -0.6])
    shifts = gen.sample_shifts(8, 2, 7, 3)
    ref, iters = O.translate_average(phase, LAME10, f, shifts, tol=1e-10)
    dt = torch.float64 if prec == "f64" else torch.float32
    plan = Plan([shape], prec=prec, max_batch=4)
    avg, reps = plan.translate_average(torch.from_numpy(phase).to(dev), LAME10,
                                       torch.from_numpy(f).to(dev).to(dt), shifts, tol=1e-10)
    a = avg.cpu().numpy()
    if prec == "f64":
        assert [r.iters for r in reps] == iters
        np.testing.assert_allclose(a, ref, atol=1e-10 * np.abs(ref).max())
    else:
        s = 3
        e_gpu, e_ref = a[4:4 + s], ref[4:4 + s]
        assert O.relative_strain_error_voigt(e_gpu, e_ref) < 1e-5
    np.testing.assert_array_equal(a[-1], ref[-1])
    plan.close()


def test_translate_average_3d_batch_groups(torch_dev):
    say("translated average 3D, two groups of different sizes")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    shapes = [(16, 16, 16), (24, 24, 24)]
    plan = Plan(shapes, prec="f64", max_batch=5)
    groups, refs = [], []
    for g, shp in enumerate(shapes):
        cell = 8
        ph = gen.tile_cell(gen.rsa_cell(cell, 3, 0.2, 1.5, 2.5, seed=g)[0], shp)
        f = gen.bump_force(shp, gen.random_center(shp, g), 4.0, gen.random_direction(3, g))
        sh = gen.sample_shifts(cell, 3, 4, g)
        groups.append(dict(grid=g, phase=torch.from_numpy(ph).to(dev), lame=LAME10,
                           f=torch.from_numpy(f).to(dev), shifts=sh))
        refs.append(O.translate_average(ph, LAME10, f, sh, tol=1e-9)[0])
    avgs, reps, st = plan.translate_average_batch(groups, tol=1e-9)
    for a, ref in zip(avgs, refs):
        np.testing.assert_allclose(a.cpu().numpy(), ref, atol=1e-10 * np.abs(ref).max())
    plan.close()


# ---------------------------------------------------------------- statuses and edge cases

def test_status_paths(torch_dev):
    say("status paths")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan, LsfftError, E_NOCONV
    shape = (16, 16)
    phase = rand_phase(shape, 31)
    f = rand_force(shape, 32)
    res, rep = gpu_solve(torch_dev, shape, phase, LAME10, f, tol=1e-12, max_iter=3)
    assert rep.status == E_NOCONV and rep.iters == 3
    # zero force: nothing to solve, zero fields
    res, rep = gpu_solve(torch_dev, shape, phase, LAME10, np.zeros((2,) + shape))
    assert rep.status == 0 and rep.iters == 0 and np.abs(res["eps"]).max() == 0.0
    # phase id outside the table
    bad = phase.copy()
    bad[3, 3] = 2
    plan = Plan([shape], prec="f64")
    with pytest.raises(LsfftError):
        plan.solve(torch.from_numpy(bad).to(dev), LAME10, torch.from_numpy(f).to(dev))
    # strict equilibrium: a one-signed bump is rejected, a dipole accepted
    plan_s = Plan([shape], prec="f64", strict_equil=True)
    bump = gen.bump_force(shape, (7.5, 7.5), 5.0, [1.0, 0.0])
    with pytest.raises(LsfftError):
        plan_s.solve(torch.from_numpy(phase).to(dev), LAME10, torch.from_numpy(bump).to(dev))
    dip = gen.dipole_force(shape, (7.5, 7.5), 4.0, [1.0, 0.0], 3)
    out, rep = plan_s.solve(torch.from_numpy(phase).to(dev), LAME10, torch.from_numpy(dip).to(dev), tol=1e-9)
    assert rep.status == 0
    plan.close()
    plan_s.close()


def test_determinism(torch_dev):
    say("bitwise determinism")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    shape = (24, 32, 16)
    phase = rand_phase(shape, 41)
    f = rand_force(shape, 42)
    for prec in ("f32", "f64"):
        dt = torch.float64 if prec == "f64" else torch.float32
        plan = Plan([shape], prec=prec)
        a, ra = plan.solve(torch.from_numpy(phase).to(dev), LAME10, torch.from_numpy(f).to(dev).to(dt), tol=1e-7)
        b, rb = plan.solve(torch.from_numpy(phase).to(dev), LAME10, torch.from_numpy(f).to(dev).to(dt), tol=1e-7)
        assert ra.iters == rb.iters and ra.residual == rb.residual
        for k in a:
            assert torch.equal(a[k], b[k])
        plan.close()


def test_timing_plan_matches_graph_plan(torch_dev):
    """The timed plan (graphs off, event pairs stamped by every launch) computes
    the same iterates bit for bit and accounts one launch of each pass class
    per iteration."""
    say("timing plan vs graph plan, 3D 16x24x32 FP32")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan, K_GREEN, K_XPASS, K_YPASS, K_REDUCE
    shape = (16, 24, 32)
    phase = rand_phase(shape, 41)
    f = torch.from_numpy(rand_force(shape, 42)).to(dev).float()
    ph = torch.from_numpy(phase).to(dev)
    outs = []
    for timing in (False, True):
        plan = Plan([shape], prec="f32", timing=timing)
        o, rep = plan.solve(ph, LAME10, f, tol=1e-6)
        torch.cuda.synchronize()
        outs.append((o["eps"].cpu(), rep.iters))
        if timing:
            for k in (K_GREEN, K_XPASS, K_YPASS, K_REDUCE):
                ms, n = plan.kernel_times(k)
                assert ms > 0.0 and n >= rep.iters, (k, ms, n, rep.iters)
        plan.close()
    assert outs[0][1] == outs[1][1]
    assert torch.equal(outs[0][0], outs[1][0])


def test_failure_injection_in_a_batch(torch_dev):
    """A NaN in one force and a far too soft reference medium in another are
    caught on the device (E_DIVERGED at the first residual, resp. when the
    residual grows) and retire alone: the healthy solves of the same batch
    equal their single solves bit for bit."""
    say("failure injection: NaN force, too soft C0, healthy neighbours")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan, E_DIVERGED
    shape = (16, 16)
    phase = rand_phase(shape, 51)
    f = rand_force(shape, 52)
    fnan = f.copy()
    fnan[0, 5, 7] = np.nan
    lam0, mu0 = O.reference_medium(LAME10)
    probs = [dict(phase=torch.from_numpy(phase).to(dev), lame=LAME10, f=torch.from_numpy(f).to(dev)),
             dict(phase=torch.from_numpy(phase).to(dev), lame=LAME10, f=torch.from_numpy(fnan).to(dev)),
             dict(phase=torch.from_numpy(phase).to(dev), lame=LAME10, f=torch.from_numpy(f).to(dev),
                  c0=(0.01 * lam0, 0.01 * mu0)),
             dict(phase=torch.from_numpy(phase).to(dev), lame=LAME10, f=torch.from_numpy(2.0 * f).to(dev))]
    plan = Plan([shape], prec="f64", max_batch=4)
    outs, reps, st = plan.solve_batch(probs, tol=1e-9, max_iter=2000)
    print("statuses", [r.status for r in reps], "iters", [r.iters for r in reps])
    assert st == E_DIVERGED
    assert reps[0].status == 0 and reps[3].status == 0
    assert reps[1].status == E_DIVERGED and reps[2].status == E_DIVERGED
    single, _ = plan.solve(probs[0]["phase"], LAME10, probs[0]["f"], tol=1e-9, max_iter=2000)
    assert torch.equal(outs[0]["eps"], single["eps"])
    plan.close()
