"""Full-size checks at the 128^3 single-solve workload (3D, 8^3 cells of
16^3, one sphere per cell vf 0.25, contrast 10, vector bump R = 12), in the
launch configuration bench.py times.

* FP64: the complete oracle solve (Algorithm 1, NumPy FP64) at full size,
  computed once per module (a few minutes of CPU), iterate count and strain
  compared to the GPU.
* FP32: relative strain error against that oracle solution <= 1e-5; with the
  FP64 defect correction (the configuration bench.py times) the
  FP64-evaluated residual meets 1e-8 and the error is <= 1e-6.  At contrast
  100 the FP32 + correction run is compared with the FP64 GPU solve (the
  oracle would need about a thousand iterations at 128^3).
* Properties that hold at any size, computed on the CPU in FP64 from the
  GPU fields: the equilibrium residual equals the reported one, sigma = L eps,
  eps = sym grad u.
"""
import sys

import numpy as np
import pytest

import gen
from oracle import lsfft_oracle as O

pytestmark = pytest.mark.gpu

SHAPE = (128, 128, 128)


def say(msg):
    print(f"\n[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    phase, _ = gen.inclusion_per_cell(SHAPE, 16, 0.25)
    f = gen.bump_force(SHAPE, gen.random_center(SHAPE, 0), 12.0, gen.random_direction(3, 1))
    lame = O.lame_from_young(gen.Material.two_phase(1.0, 10.0).table())
    return torch, torch.device("cuda:0"), phase, f, lame


@pytest.fixture(scope="module")
def gpu_results(setup):
    torch, dev, phase, f, lame = setup
    from paper_2601_00822_amd import Plan
    out = {}
    for prec, dt, refine in (("f64", torch.float64, False), ("f32", torch.float32, False),
                             ("f32r", torch.float32, True)):
        say(f"128^3 solve {prec}")
        plan = Plan([SHAPE], prec=prec[:3], refine=refine)
        res, rep = plan.solve(torch.from_numpy(phase).to(dev), lame, torch.from_numpy(f).to(dev).to(dt), tol=1e-8)
        torch.cuda.synchronize()
        out[prec] = ({k: v.double().cpu().numpy() for k, v in res.items()}, rep)
        plan.close()
    return out


@pytest.fixture(scope="module")
def oracle128(setup):
    """The oracle's solution of the 128^3 workload at 1e-8."""
    torch, dev, phase, f, lame = setup
    say("oracle full solve at 128^3 (CPU, a few minutes)")
    ref = O.solve_basic(phase, lame, f, tol=1e-8)
    return ref


def independent_residual(phase, lame, f, sig):
    """||div sigma + P f|| / ||P f|| from the real stress field, in FP64."""
    shape = phase.shape
    xi = O.wavevectors(shape)
    w = O.hermitian_weights(shape)
    s_hat = O.fft_r(O.from_voigt(sig, 3), shape)
    f_hat = O.fft_r(f, shape)
    f_hat[:, O.zero_set(shape)] = 0.0
    r = O.div_hat(s_hat, xi) + f_hat
    return float(np.sqrt(np.sum(w * np.abs(r) ** 2) / np.sum(w * np.abs(f_hat) ** 2)))


def test_fp64_properties(setup, gpu_results):
    torch, dev, phase, f, lame = setup
    res, rep = gpu_results["f64"]
    say(f"fp64 properties iters={rep.iters} residual={rep.residual:.3e}")
    assert rep.status == 0 and rep.residual <= 1e-8
    r = independent_residual(phase, lame, f, res["sig"])
    assert abs(r - rep.residual) <= 1e-3 * rep.residual, (r, rep.residual)
    lam, mu = O.field_moduli(phase, lame)
    e = O.from_voigt(res["eps"], 3)
    np.testing.assert_allclose(O.to_voigt(O.stress(e, lam, mu)), res["sig"], atol=1e-12 * np.abs(res["sig"]).max())
    xi = O.wavevectors(SHAPE)
    e_from_u = O.ifft_r(O.sym_grad_hat(O.fft_r(res["u"], SHAPE), xi), SHAPE)
    assert O.relative_strain_error(e_from_u, e) < 1e-10


def test_fp32_against_oracle(setup, gpu_results, oracle128):
    torch, dev, phase, f, lame = setup
    r32, rep32 = gpu_results["f32"]
    err = O.relative_strain_error_voigt(r32["eps"], O.to_voigt(oracle128.eps))
    r = independent_residual(phase, lame, f, r32["sig"])
    say(f"fp32 status={rep32.status} iters={rep32.iters} residual={rep32.residual:.3e} "
        f"cpu residual={r:.3e} strain err vs oracle={err:.3e}")
    assert rep32.status in (0, 1)
    assert err < 1e-5
    assert abs(r - rep32.residual) <= 0.05 * rep32.residual


def test_fp64_against_full_oracle(setup, gpu_results, oracle128):
    torch, dev, phase, f, lame = setup
    res, rep = gpu_results["f64"]
    ref = oracle128
    err = O.relative_strain_error_voigt(res["eps"], O.to_voigt(ref.eps))
    print(f"oracle iters={ref.iters} gpu iters={rep.iters} err={err:.3e}", flush=True)
    assert rep.iters == ref.iters
    assert err < 1e-10
    assert np.abs(res["u"] - ref.u).max() < 1e-10 * np.abs(ref.u).max()


def test_fp32_refined_against_oracle(setup, gpu_results, oracle128):
    torch, dev, phase, f, lame = setup
    r32, rep = gpu_results["f32r"]
    err = O.relative_strain_error_voigt(r32["eps"], O.to_voigt(oracle128.eps))
    serr = O.relative_strain_error_voigt(r32["sig"], O.to_voigt(oracle128.sig))
    r = independent_residual(phase, lame, f, r32["sig"])
    say(f"fp32+fp64 correction iters={rep.iters} residual={rep.residual:.3e} cpu residual of the fp32 "
        f"fields={r:.3e} strain err vs oracle={err:.3e} stress err={serr:.3e}")
    assert rep.status == 0 and rep.residual <= 1e-8
    assert err < 1e-6 and serr < 1e-5


@pytest.mark.parametrize("scheme", ["basic", "cg"])
def test_refined_high_contrast_128(setup, scheme):
    """128^3, random spheres vf 0.3 (r 3-6) in 16^3 cells, contrast 100, bump
    R = 12: FP32 with the FP64 correction against the FP64 basic solve."""
    torch, dev, _, _, _ = setup
    from paper_2601_00822_amd import Plan
    say(f"128^3 contrast 100 FP32+FP64 correction, {scheme}")
    phase = gen.tile_cell(gen.rsa_cell(16, 3, 0.3, 3.0, 6.0, seed=11)[0], SHAPE)
    f = gen.bump_force(SHAPE, gen.random_center(SHAPE, 5), 12.0, gen.random_direction(3, 6))
    lame = O.lame_from_young(gen.Material.two_phase(1.0, 100.0).table())
    ph, fd = torch.from_numpy(phase).to(dev), torch.from_numpy(f).to(dev)
    p64 = Plan([SHAPE], prec="f64")
    o64, r64 = p64.solve(ph, lame, fd, tol=1e-8, max_iter=20000)
    p64.close()
    p32 = Plan([SHAPE], prec="f32", scheme=scheme, refine=True)
    o32, r32 = p32.solve(ph, lame, fd.float(), tol=1e-8, max_iter=20000)
    p32.close()
    e = O.relative_strain_error_voigt(o32["eps"].double().cpu().numpy(), o64["eps"].cpu().numpy())
    print(f"fp64 iters {r64.iters}; fp32 {scheme} iters {r32.iters} residual {r32.residual:.3e} err {e:.3e}")
    assert r64.status == 0 and r32.status == 0 and r32.residual <= 1e-8
    assert e < 1e-6
