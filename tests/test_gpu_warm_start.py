"""Warm starts of lsfft_solve_bfcs: the iteration begins at a given
displacement (its spectrum projected off the xi = 0 set) instead of the free
term; parity with the oracle's displacement-form iteration from the same
start.  Every test prints its case before the first GPU call."""
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


@pytest.mark.parametrize("shape", [(32, 32), (12, 16, 8)])
def test_fp64_warm_start_matches_oracle(torch_dev, shape):
    say(f"warm start FP64 {shape}, batch of 3 in chunks of 2")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    d = len(shape)
    probs, refs = [], []
    for k in range(3):
        ph = (np.random.default_rng(80 + k).random(shape) < 0.35).astype(np.uint8)
        f = np.random.default_rng(90 + k).normal(size=(d,) + shape)
        u0 = np.random.default_rng(100 + k).normal(size=(d,) + shape) * 0.3 + 2.0
        refs.append(O.solve_displacement_update(ph, LAME, f, tol=1e-9, u_init=u0))
        probs.append(dict(phase=torch.from_numpy(ph).to(dev), lame=LAME, f=torch.from_numpy(f).to(dev),
                          u0=torch.from_numpy(u0).to(dev)))
    plan = Plan([shape], prec="f64", max_batch=2)
    outs, reps, _ = plan.solve_batch(probs, tol=1e-9)
    plan.close()
    for o, r, ref in zip(outs, reps, refs):
        print("iters", r.iters, ref.iters)
        assert r.iters == ref.iters
        e = O.relative_strain_error_voigt(o["eps"].cpu().numpy(), O.to_voigt(ref.eps))
        eu = np.linalg.norm(o["u"].cpu().numpy() - ref.u) / np.linalg.norm(ref.u)
        assert e < 1e-10 and eu < 1e-10, (e, eu)


def test_fp32_warm_start_from_the_solution(torch_dev):
    say("warm start FP32 3D 16^3 from the FP64 solution")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    shape = (16, 16, 16)
    ph = (np.random.default_rng(110).random(shape) < 0.35).astype(np.uint8)
    f = np.random.default_rng(111).normal(size=(3,) + shape)
    ref = O.solve_basic(ph, LAME, f, tol=1e-10)
    plan = Plan([shape], prec="f32")
    cold, rc = plan.solve(torch.from_numpy(ph).to(dev), LAME, torch.from_numpy(f).to(dev).float(), tol=1e-5)
    warm, rw = plan.solve(torch.from_numpy(ph).to(dev), LAME, torch.from_numpy(f).to(dev).float(), tol=1e-5,
                          u0=torch.from_numpy(ref.u).to(dev).float())
    plan.close()
    print("cold", rc.iters, "warm", rw.iters, rw.residual)
    assert rw.status == 0 and rw.iters < rc.iters
    assert O.relative_strain_error_voigt(warm["eps"].cpu().numpy(), O.to_voigt(ref.eps)) < 1e-5


def test_warm_start_argument_checks(torch_dev):
    say("warm start argument checks (CG, FP64 correction, partial starts)")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan, LsfftError
    shape = (16, 16)
    ph = torch.zeros(shape, dtype=torch.uint8, device=dev)
    f = torch.from_numpy(np.random.default_rng(120).normal(size=(2,) + shape)).to(dev)
    u0 = torch.zeros((2,) + shape, dtype=torch.float64, device=dev)
    plan = Plan([shape], prec="f64", scheme="cg")
    with pytest.raises(LsfftError):
        plan.solve(ph, LAME, f, u0=u0)
    plan.close()
    plan = Plan([shape], prec="f32", refine=True)
    with pytest.raises(LsfftError):
        plan.solve(ph, LAME, f.float(), u0=u0.float())
    plan.close()
    plan = Plan([shape], prec="f64", max_batch=2)
    with pytest.raises(ValueError):
        plan.solve_batch([dict(phase=ph, lame=LAME, f=f, u0=u0), dict(phase=ph, lame=LAME, f=f)])
    plan.close()
