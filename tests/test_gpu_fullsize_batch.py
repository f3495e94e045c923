"""Full-size checks of the batched translated-averaging workload the benchmark
times (512 solves: eight groups of 64 intra-cell shifts on 48^3, 64^3 and
96^3 grids, RSA spheres, contrasts 2-100, tol 1e-8), in its launch
configuration: one batch of all 512 solves, FP32 inner solves with the FP64
defect correction, schedule variants tuned on the plan's grids.

At these sizes the oracle would need tens of thousands of FP64 solves, so the
averages are checked through identities that every shifted solve satisfies
and that averaging keeps, evaluated on the host in FP64 with the oracle's
transforms (Eqs. 3.3-3.6: the average of fields, of fields times the
inclusion indicator V, and of V):

* <V> equals the average of the shifted indicators, exactly (64 shifts);
* compatibility: <eps> = sym grad <u>;
* the two-phase constitutive split: <sigma> = L_m <eps> + (L_i - L_m) <eps V>
  and <sigma V> = L_i <eps V>;
* equilibrium: div <sigma> + P f = 0.

The solves stop at an FP64 residual of 1e-8 and their fields are then
materialized in FP32 from the rounded state, so the identities hold to FP32
rounding (measured: constitutive split 1e-15, compatibility up to 6e-7,
equilibrium up to 4e-6, whose high wavenumbers amplify the rounding of
sigma; bars 1e-6, 2e-6 and 2e-5); a wrong tile, shift or phase map breaks
them by orders of magnitude more.
"""
import sys

import numpy as np
import pytest

import bench
from oracle import lsfft_oracle as O

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"\n[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def batch_results():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_00822_amd import Plan, lame_from_young
    dev = torch.device("cuda:0")
    groups = bench.make_batch(0)
    shapes = sorted({g["shape"] for g in groups})
    dgroups = [dict(grid=shapes.index(g["shape"]), phase=torch.from_numpy(g["phase"]).to(dev),
                    lame=lame_from_young(g["table"]), f=torch.from_numpy(g["f"]).to(dev).float(),
                    shifts=g["shifts"]) for g in groups]
    nsolve = sum(len(g["shifts"]) for g in groups)
    say(f"batch of {nsolve} solves on {shapes}, FP32 + FP64 correction, tuned")
    plan = Plan(shapes, prec="f32", max_batch=nsolve, refine=True)
    plan.autotune(iters=20)
    avgs, reps, st = plan.translate_average_batch(dgroups, tol=1e-8)
    torch.cuda.synchronize()
    out = [a.cpu().numpy() for a in avgs]
    plan.close()
    return groups, out, reps, st


def split(avg, d):
    s = len(O.VOIGT[d])
    k = 0
    parts = {}
    for name, n in (("u", d), ("uV", d), ("eps", s), ("epsV", s), ("sig", s), ("sigV", s), ("V", 1)):
        parts[name] = avg[k:k + n]
        k += n
    return parts


def test_every_solve_converged(batch_results):
    groups, avgs, reps, st = batch_results
    say("batch status and per-solve FP64 residuals")
    assert st == 0
    assert len(reps) == sum(len(g["shifts"]) for g in groups)
    worst = max(r.residual for r in reps)
    print(f"statuses {sorted({r.status for r in reps})}, worst residual {worst:.3e}, "
          f"iterations {min(r.iters for r in reps)}-{max(r.iters for r in reps)}")
    assert all(r.status == 0 for r in reps)
    assert worst <= 1e-8


@pytest.mark.parametrize("gi", range(8))
def test_group_average_identities(batch_results, gi):
    groups, avgs, reps, st = batch_results
    g = groups[gi]
    shape = g["shape"]
    d = 3
    say(f"group {gi}: {shape}, contrast {g['contrast']:.1f}, {len(g['shifts'])} shifts")
    p = split(avgs[gi], d)
    # <V>: the average of the shifted inclusion indicators, exact
    ind = np.zeros(shape)
    for chi in np.asarray(g["shifts"]).reshape(-1, d):
        ind += np.roll(g["phase"] == 1, shift=tuple(int(c) for c in chi), axis=(0, 1, 2))
    np.testing.assert_array_equal(p["V"][0], ind / len(g["shifts"]))
    # compatibility of the averaged fields
    xi = O.wavevectors(shape)
    e_from_u = O.ifft_r(O.sym_grad_hat(O.fft_r(p["u"], shape), xi), shape)
    comp = O.relative_strain_error(e_from_u, O.from_voigt(p["eps"], d))
    # the constitutive split over the two phases
    (lam_m, mu_m), (lam_i, mu_i) = O.lame_from_young(np.asarray(g["table"]))[:2]
    eps, epsv = O.from_voigt(p["eps"], d), O.from_voigt(p["epsV"], d)
    sig_pred = O.stress(eps, lam_m, mu_m) + O.stress(epsv, lam_i - lam_m, mu_i - mu_m)
    sigv_pred = O.stress(epsv, lam_i, mu_i)
    scale = np.abs(p["sig"]).max()
    c1 = np.abs(O.to_voigt(sig_pred) - p["sig"]).max() / scale
    c2 = np.abs(O.to_voigt(sigv_pred) - p["sigV"]).max() / scale
    # equilibrium of the averaged stress with the (projected) force
    w = O.hermitian_weights(shape)
    f_hat = O.fft_r(np.asarray(g["f"], dtype=np.float32).astype(np.float64), shape)   # the force the plan sees
    f_hat[:, O.zero_set(shape)] = 0.0
    r = O.div_hat(O.fft_r(O.from_voigt(p["sig"], d), shape), xi) + f_hat
    res = float(np.sqrt(np.sum(w * np.abs(r) ** 2) / np.sum(w * np.abs(f_hat) ** 2)))
    print(f"compatibility {comp:.2e}, constitutive {c1:.2e} / {c2:.2e}, equilibrium {res:.2e}")
    assert comp < 2e-6
    assert c1 < 1e-6 and c2 < 1e-6
    assert res < 2e-5
