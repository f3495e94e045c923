"""GPU parity of the RVE identification (Definition 2.2) against the oracle,
and the enlargement of the body-force unit cell.  Every test prints its case
before the first GPU call."""
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


def test_profile_of_random_fields_matches_oracle(torch_dev):
    say("RVE radial maxima of random fields, 3D 8x12x16 and 2D 24x16 with spacing")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    rng = np.random.default_rng(5)
    for shape, center, h in [((8, 12, 16), (3.5, 11.0, 0.25), None), ((24, 16), (7.0, 15.5), (0.5, 2.0))]:
        d = len(shape)
        s = 6 if d == 3 else 3
        avg = rng.normal(size=(2 * d + 4 * s + 1,) + shape) * np.exp(rng.normal(size=shape))
        plan = Plan([shape], prec="f64", spacing=None if h is None else [h])
        got = plan.rve_identify(torch.from_numpy(avg).to(dev), center, 2.0, tol=0.3, dr=0.7)
        plan.close()
        radius, fits, pe, ps = O.rve_radius(avg, center, 2.0, 0.3, h=h, dr=0.7)
        np.testing.assert_array_equal(got["profile_eps"], pe)
        np.testing.assert_array_equal(got["profile_sig"], ps)
        assert got["radius"] == radius and got["fits"] == fits


def test_translated_average_rve_matches_oracle(torch_dev):
    say("RVE of a translated average, 2D 32x32 dipole")
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    shape = (32, 32)
    cell, _ = gen.inclusion_per_cell((8, 8), 8, 0.25)
    phase = gen.tile_cell(cell, shape)
    f = gen.dipole_force(shape, (16.0, 16.0), 2.5, [1.0, 0.0], 2)
    shifts = gen.all_shifts(8, 2)
    plan = Plan([shape], prec="f64", max_batch=64)
    avg, _ = plan.translate_average(torch.from_numpy(phase).to(dev), LAME, torch.from_numpy(f).to(dev), shifts,
                                    tol=1e-10)
    got = plan.rve_identify(avg, (16.0, 16.0), 4.5, tol=5e-2)
    plan.close()
    radius, fits, pe, ps = O.rve_radius(avg.cpu().numpy(), (16.0, 16.0), 4.5, 5e-2)
    print("radius", got["radius"], "fits", got["fits"])
    np.testing.assert_array_equal(got["profile_eps"], pe)
    assert got["radius"] == radius and got["fits"] == fits
    # the averaged fields decay: the profile falls by the tolerance by the RVE edge
    assert np.isfinite(radius) and pe[int(radius):].max() < 5e-2 * pe.max()


def test_bfuc_enlargement(torch_dev):
    say("BFUC enlargement, 2D cell 8, dipole, from 2 cells per axis")
    torch, dev = torch_dev
    from paper_2601_00822_amd.rve import find_bfuc
    cell, _ = gen.inclusion_per_cell((8, 8), 8, 0.25)

    def force_at(shape, center):
        return gen.dipole_force(shape, center, 2.5, [1.0, 0.0], 2)

    res = find_bfuc(cell, LAME, force_at, 4.5, gen.all_shifts(8, 2), tol=3e-2, cells=2, max_len=256,
                    prec="f64", solve_tol=1e-10, printer=print)
    assert res["found"]
    sizes = [h[0][0] for h in res["history"]]
    assert sizes[0] == 16 and len(sizes) >= 2          # the smallest cell is too small
    assert not res["history"][0][1]["fits"]
    info = res["rve"]
    assert info["radius"] + 2.25 <= info["box_radius"]
    # Definition 2.2: inside the RVE the averaged strain no longer depends on
    # the size of the BFUC (to the tolerance): compare with the next size up
    L = res["shape"][0]
    bigger = [n for n in (24, 32, 48, 64, 96, 128, 256) if n > L and n % 8 == 0][0]
    res2 = find_bfuc(cell, LAME, force_at, 4.5, gen.all_shifts(8, 2), tol=3e-2, cells=bigger // 8,
                     max_len=bigger, prec="f64", solve_tol=1e-10)
    a = res["avg"].cpu().numpy()
    b = res2["avg"].cpu().numpy()
    off = (bigger - L) // 2
    b = b[:, off:off + L, off:off + L]
    yy, xx = np.meshgrid(np.arange(L) - L / 2, np.arange(L) - L / 2, indexing="ij")
    inside = np.sqrt(yy ** 2 + xx ** 2) < info["radius"]
    ea, eb = a[4:7][:, inside], b[4:7][:, inside]
    rel = np.linalg.norm(ea - eb) / np.linalg.norm(eb)
    print("BFUC", L, "vs", bigger, "strain inside the RVE differs by", rel)
    assert rel < 5e-2
