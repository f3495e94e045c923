"""GPU check of the surrogate's dataset construction: the averaged strain
obtained by convolving a force with the averaged point-force kernel (three
translate_average calls of the FP64 solver) equals the solver's direct
translation average of that force over every shift of the cell."""
import sys

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


def test_kernel_convolution_equals_direct_average():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_00822_amd import Plan, lame_from_young
    from paper_2601_00822_amd import surrogate as S
    print("\n[case] averaged-strain kernel 32^3, cell 8, 512 shifts, FP64", flush=True)
    sys.stdout.flush()
    n, cell = 32, 8
    dev = torch.device("cuda:0")
    phase_np = gen.tile_cell(gen.rsa_cell(cell, 3, 0.2, 1.5, 2.5, seed=4)[0], (n, n, n))
    phase = torch.from_numpy(phase_np).to(dev)
    lame = lame_from_young(gen.Material.two_phase(1.0, 10.0).table())
    K, reps = S.averaged_strain_kernel(phase, lame, cell, prec="f64", max_batch=256, tol=1e-10)
    assert all(r.status == 0 for r in reps)
    f = gen.bump_set_torch(n, gen.bump_set_params(n, 1, seed=7, rmin=3.0, rmax=6.0), dev)
    conv = S.averaged_strain_from_kernel(S.kernel_spectrum(K), f)[0]
    plan = Plan([(n, n, n)], prec="f64", max_batch=256)
    avg, _ = plan.translate_average(phase, lame, f[0].contiguous(), S.cell_shifts(cell), tol=1e-10)
    plan.close()
    direct = avg[6:12]
    err = float(torch.linalg.norm(conv - direct) / torch.linalg.norm(direct))
    print(f"kernel convolution vs direct average: {err:.2e}")
    assert err < 1e-8
    c2, d2 = S.restrict2(conv), S.restrict2(direct)
    assert c2.shape == (6, 16, 16, 16)
    assert float(torch.linalg.norm(c2 - d2) / torch.linalg.norm(d2)) < 1e-8
