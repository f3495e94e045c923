"""GPU checks of the surrogate's dataset construction, all through the
library: the kernel convolution (lsfft_kernel_convolve) against the oracle's
convolution element by element, the averaged point-force kernel of the GPU
solver against the oracle's, the convolution of a force with that kernel
against the solver's direct translation average over every shift, and the
data kernels (block means, per-sample norms, bump forces) against their
plain definitions.  Every test prints its case before the first GPU call."""
import sys

import numpy as np
import pytest

import gen
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


@pytest.mark.parametrize("shape,prec", [((16, 24, 32), "f64"), ((16, 24, 32), "f32"), ((48, 64, 8), "f64"),
                                        ((12, 32), "f64")])
def test_kernel_convolve_matches_the_oracle(torch_dev, shape, prec):
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    say(f"kernel convolution {shape} {prec}")
    d = len(shape)
    s = 6 if d == 3 else 3
    rng = np.random.default_rng(5)
    K = rng.normal(size=(s, d) + shape)
    F = rng.normal(size=(3, d) + shape)
    dt = torch.float64 if prec == "f64" else torch.float32
    if prec == "f32":
        K = K.astype(np.float32).astype(np.float64)
        F = F.astype(np.float32).astype(np.float64)
    plan = Plan([shape], prec=prec, max_batch=2)       # three forces: two batches
    out = plan.kernel_convolve(torch.from_numpy(K).to(dev).to(dt), torch.from_numpy(F).to(dev).to(dt))
    torch.cuda.synchronize()
    plan.close()
    got = out.double().cpu().numpy()
    tol = 1e-12 if prec == "f64" else 2e-6
    for b in range(3):
        want = O.kernel_convolve(K, F[b])
        scale = np.abs(want).max()
        np.testing.assert_allclose(got[b], want, rtol=0, atol=tol * scale, err_msg=f"force {b}")


def test_averaged_kernel_matches_the_oracle(torch_dev):
    """The averaged point-force strain kernel from the GPU solver's
    translated averages (FP64) equals the oracle's literal translated
    averages of the same point forces, on an 8^3 grid of 4^3 cells."""
    torch, dev = torch_dev
    from paper_2601_00822_amd import lame_from_young
    from paper_2601_00822_amd import surrogate as S
    say("averaged point-force kernel 8^3, cell 4, vs oracle")
    n, cell = 8, 4
    phase_np = gen.tile_cell(gen.rsa_cell(cell, 3, 0.25, 0.8, 1.2, seed=2)[0], (n, n, n))
    lame = lame_from_young(gen.Material.two_phase(1.0, 10.0).table())
    K, reps = S.averaged_strain_kernel(torch.from_numpy(phase_np).to(dev), lame, cell, prec="f64", max_batch=64,
                                       tol=1e-11)
    assert all(r.status == 0 for r in reps)
    got = K.cpu().numpy()
    shifts = gen.all_shifts(cell, 3)
    for j in range(3):
        delta = gen.point_force((n, n, n), j)
        avg, _ = O.translate_average(phase_np, lame, delta, shifts, tol=1e-11)
        want = avg[6:12]
        np.testing.assert_allclose(got[:, j], want, rtol=0, atol=1e-9 * np.abs(want).max(), err_msg=f"axis {j}")


def test_kernel_convolution_equals_direct_average(torch_dev):
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan, lame_from_young, bump_forces, block_mean
    from paper_2601_00822_amd import surrogate as S
    say("averaged-strain kernel 32^3, cell 8, 512 shifts, FP64; library convolution vs direct average")
    n, cell = 32, 8
    phase_np = gen.tile_cell(gen.rsa_cell(cell, 3, 0.2, 1.5, 2.5, seed=4)[0], (n, n, n))
    phase = torch.from_numpy(phase_np).to(dev)
    lame = lame_from_young(gen.Material.two_phase(1.0, 10.0).table())
    K, reps = S.averaged_strain_kernel(phase, lame, cell, prec="f64", max_batch=256, tol=1e-10)
    assert all(r.status == 0 for r in reps)
    f = bump_forces((n, n, n), gen.bump_set_params(n, 1, seed=7, rmin=3.0, rmax=6.0))
    conv = S.averaged_strain_from_kernel(K, f)[0]
    plan = Plan([(n, n, n)], prec="f64", max_batch=256)
    avg, _ = plan.translate_average(phase, lame, f[0].contiguous(), S.cell_shifts(cell), tol=1e-10)
    plan.close()
    direct = avg[6:12].contiguous()
    c, dr = conv.cpu().numpy(), direct.cpu().numpy()
    err = np.linalg.norm(c - dr) / np.linalg.norm(dr)
    print(f"kernel convolution vs direct average: {err:.2e}")
    assert err < 1e-8
    np.testing.assert_allclose(c, dr, rtol=0, atol=1e-8 * np.abs(dr).max())
    c2, d2 = block_mean(conv.contiguous(), 2).cpu().numpy(), block_mean(direct, 2).cpu().numpy()
    assert c2.shape == (6, 16, 16, 16)
    assert np.linalg.norm(c2 - d2) / np.linalg.norm(d2) < 1e-8


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_data_kernels(torch_dev, prec):
    """Block means and scaled copies, per-sample norms and bump forces
    against their plain definitions (numpy block reshapes, numpy norms, the
    input generator's bump force)."""
    torch, dev = torch_dev
    from paper_2601_00822_amd import block_mean, sample_norms, relative_l2, bump_forces
    say(f"data kernels {prec}")
    dt = torch.float64 if prec == "f64" else torch.float32
    tol = 1e-14 if prec == "f64" else 1e-6
    rng = np.random.default_rng(11)
    a = rng.normal(size=(3, 2, 8, 12, 16))
    got = block_mean(torch.from_numpy(a).to(dev).to(dt), 2, scale=3.0).double().cpu().numpy()
    want = 3.0 * a.reshape(3, 2, 4, 2, 6, 2, 8, 2).mean(axis=(3, 5, 7))
    np.testing.assert_allclose(got, want, rtol=tol, atol=tol)
    a2 = rng.normal(size=(4, 6, 10))
    got2 = block_mean(torch.from_numpy(a2).to(dev).to(dt), 2, spatial=2).double().cpu().numpy()
    np.testing.assert_allclose(got2, a2.reshape(4, 3, 2, 5, 2).mean(axis=(2, 4)), rtol=tol, atol=tol)
    got3 = block_mean(torch.from_numpy(a).to(dev).to(dt), 1, scale=0.5).double().cpu().numpy()
    np.testing.assert_allclose(got3, 0.5 * a, rtol=tol, atol=tol)
    if prec == "f64":   # rounded once to FP32 on the way out
        got4 = block_mean(torch.from_numpy(a).to(dev), 2, dtype=torch.float32).cpu().numpy()
        np.testing.assert_allclose(got4, (want / 3.0).astype(np.float32), rtol=1e-7, atol=1e-7)
    t = rng.normal(size=(5, 3, 7, 9))
    y = t + 0.01 * rng.normal(size=t.shape)
    tt, yy = torch.from_numpy(t).to(dev).to(dt), torch.from_numpy(y).to(dev).to(dt)
    nd, nt = sample_norms(tt, yy)
    tq, yq = tt.double().cpu().numpy(), yy.double().cpu().numpy()
    np.testing.assert_allclose(nt, np.linalg.norm(tq.reshape(5, -1), axis=1), rtol=1e-13)
    np.testing.assert_allclose(nd, np.linalg.norm((yq - tq).reshape(5, -1), axis=1), rtol=1e-12)
    np.testing.assert_allclose(relative_l2(yy, tt), nd / nt, rtol=0, atol=0)
    n0, _ = sample_norms(tt)
    np.testing.assert_allclose(n0, nt, rtol=0, atol=0)
    for shape in [(16, 12, 20), (24, 18)]:
        d = len(shape)
        params = [[(np.array([3.3, 11.9, 19.5][:d]), 6.5, gen.random_direction(d, 3)),
                   (np.array([0.2, 5.0, 7.7][:d]), 3.0, gen.random_direction(d, 4))],
                  [(np.array([8.0, 0.0, 10.0][:d]), 9.5, gen.random_direction(d, 5))]]
        got = bump_forces(shape, params, dtype=dt).double().cpu().numpy()
        for i, bumps in enumerate(params):
            want = sum(gen.bump_force(shape, c, r, v) for c, r, v in bumps)
            np.testing.assert_allclose(got[i], want, rtol=0, atol=tol * np.abs(want).max())
