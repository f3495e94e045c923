"""Full-size checks at the 256^3 workload the benchmark times (3D, 16^3
cells of 16^3, RSA spheres vf 0.3 r 3-6, stiff inclusions contrast 100,
vector bump R = 12, tol 1e-8), in its launch configuration: FP32 inner
solves with the FP64 defect correction on an autotuned plan.

At contrast 100 the oracle needs about a thousand iterations of a 256^3
grid (hours of CPU), so the fields are checked through properties that
hold at any size, computed on the host in FP64 with the oracle's transforms
from the fields the GPU returns:

* FP64 plan: the equilibrium residual recomputed from the returned stress
  equals the reported one (and is at most 1e-8); sigma = L(x) eps voxel by
  voxel; eps = sym grad u.  Together these make the FP64 fields the
  discrete solution to the tolerance, independently of the GPU's own
  residual.
* FP32 + FP64 correction: the FP64-evaluated residual meets 1e-8, the
  strain and stress agree with that verified FP64 solution to 1e-6 and
  1e-5, and the returned FP32 fields satisfy Hooke's law and compatibility
  at the FP32 level.
"""
import sys

import numpy as np
import pytest

import bench
from oracle import lsfft_oracle as O

pytestmark = pytest.mark.gpu

WL = bench.WORKLOADS["bfcs256"]
SHAPE = WL["shape"]


def say(msg):
    print(f"\n[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_00822_amd import lame_from_young
    phase, f, table, _ = bench.make_inputs(WL)
    return torch, torch.device("cuda:0"), phase, f, lame_from_young(table)


@pytest.fixture(scope="module")
def gpu_results(setup):
    torch, dev, phase, f, lame = setup
    from paper_2601_00822_amd import Plan
    out = {}
    for prec, dt, refine in (("f64", torch.float64, False), ("f32r", torch.float32, True)):
        say(f"256^3 contrast-100 solve {prec}")
        plan = Plan([SHAPE], prec=prec[:3], refine=refine)
        if prec == "f32r":
            plan.autotune(iters=20)
        res, rep = plan.solve(torch.from_numpy(phase).to(dev), lame, torch.from_numpy(f).to(dev).to(dt), tol=1e-8)
        torch.cuda.synchronize()
        out[prec] = ({k: v.double().cpu().numpy() for k, v in res.items()}, rep)
        plan.close()
        del res
    return out


def independent_residual(phase, lame, f, sig):
    """||div sigma + P f|| / ||P f|| from the real stress field, in FP64."""
    shape = phase.shape
    xi = O.wavevectors(shape)
    w = O.hermitian_weights(shape)
    f_hat = O.fft_r(f, shape)
    f_hat[:, O.zero_set(shape)] = 0.0
    r = O.div_hat(O.fft_r(O.from_voigt(sig, 3), shape), xi) + f_hat
    return float(np.sqrt(np.sum(w * np.abs(r) ** 2) / np.sum(w * np.abs(f_hat) ** 2)))


def compatibility_error(eps, u):
    xi = O.wavevectors(SHAPE)
    e_from_u = O.ifft_r(O.sym_grad_hat(O.fft_r(u, SHAPE), xi), SHAPE)
    return O.relative_strain_error(e_from_u, O.from_voigt(eps, 3))


def test_fp64_256_properties(setup, gpu_results):
    torch, dev, phase, f, lame = setup
    res, rep = gpu_results["f64"]
    say(f"256^3 fp64 properties: iters={rep.iters} residual={rep.residual:.3e}")
    assert rep.status == 0 and rep.residual <= 1e-8
    r = independent_residual(phase, lame, f, res["sig"])
    print(f"host residual from the stress field: {r:.4e}", flush=True)
    assert abs(r - rep.residual) <= 1e-3 * rep.residual, (r, rep.residual)
    lam, mu = O.field_moduli(phase, lame)
    np.testing.assert_allclose(O.to_voigt(O.stress(O.from_voigt(res["eps"], 3), lam, mu)), res["sig"], rtol=0,
                               atol=1e-12 * np.abs(res["sig"]).max())
    assert compatibility_error(res["eps"], res["u"]) < 1e-10


def test_fp32_refined_256_against_the_verified_fp64_solution(setup, gpu_results):
    torch, dev, phase, f, lame = setup
    r64, _ = gpu_results["f64"]
    r32, rep = gpu_results["f32r"]
    err = O.relative_strain_error_voigt(r32["eps"], r64["eps"])
    serr = O.relative_strain_error_voigt(r32["sig"], r64["sig"])
    r = independent_residual(phase, lame, f, r32["sig"])
    say(f"256^3 fp32 + fp64 correction: iters={rep.iters} residual={rep.residual:.3e}; host residual of the "
        f"fp32 fields {r:.3e}; strain err {err:.3e}, stress err {serr:.3e} against the fp64 solution")
    assert rep.status == 0 and rep.residual <= 1e-8
    assert err < 1e-6 and serr < 1e-5
    lam, mu = O.field_moduli(phase, lame)
    np.testing.assert_allclose(O.to_voigt(O.stress(O.from_voigt(r32["eps"], 3), lam, mu)), r32["sig"], rtol=0,
                               atol=2e-6 * np.abs(r32["sig"]).max())
    assert compatibility_error(r32["eps"], r32["u"]) < 1e-5


@pytest.mark.parametrize("scheme", ["cg", "cg_plain", "anderson"])
def test_other_schemes_256_against_the_verified_fp64_solution(setup, gpu_results, scheme):
    """The Krylov and accelerated schemes at the full 256^3 contrast-100 size
    (FP32 inner solves with the FP64 correction, default schedules): FP64
    residual <= 1e-8 as reported and as recomputed on the host from the
    returned stress (to the FP32 rounding of the field), strain within 1e-6
    of the basic scheme's verified FP64 solution."""
    torch, dev, phase, f, lame = setup
    from paper_2601_00822_amd import Plan
    r64, _ = gpu_results["f64"]
    say(f"256^3 contrast-100 solve, scheme {scheme}, fp32 + fp64 correction")
    plan = Plan([SHAPE], prec="f32", refine=True, scheme=scheme)
    res, rep = plan.solve(torch.from_numpy(phase).to(dev), lame, torch.from_numpy(f).to(dev).float(), tol=1e-8)
    torch.cuda.synchronize()
    out = {k: v.double().cpu().numpy() for k, v in res.items()}
    plan.close()
    err = O.relative_strain_error_voigt(out["eps"], r64["eps"])
    r = independent_residual(phase, lame, f, out["sig"])
    print(f"{scheme}: status={rep.status} iters={rep.iters} residual={rep.residual:.3e}; host residual of the "
          f"fp32 fields {r:.3e}; strain err {err:.3e} against the fp64 basic solution", flush=True)
    assert rep.status == 0 and rep.residual <= 1e-8
    assert err < 1e-6
    assert r < 2e-4
