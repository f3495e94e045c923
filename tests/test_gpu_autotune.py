"""GPU checks of the schedule variants and the autotuner of the batched FFT
passes: every compiled variant of every pass, forced on a plan, solves like
the FP64 oracle within the FP32 bar; a tuned plan (and a plan built from the
tuner's cache file) solves like the oracle too.  Every test prints its case
before the first GPU call."""
import json
import os
import sys

import numpy as np
import pytest

import gen
from oracle import lsfft_oracle as O

pytestmark = pytest.mark.gpu

LAME10 = O.lame_from_young(gen.Material.two_phase(1.0, 10.0).table())
LONG = (48, 64, 96, 128, 256)


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


def problem(shape, seed):
    rng = np.random.default_rng(seed)
    phase = (rng.random(shape) < 0.3).astype(np.uint8)
    f = gen.bump_force(shape, gen.random_center(shape, seed + 1), 3.0, gen.random_direction(3, seed + 2))
    return phase, f.astype(np.float32).astype(np.float64)


_REF = {}


def reference(shape, seed):
    key = (shape, seed)
    if key not in _REF:
        phase, f = problem(shape, seed)
        _REF[key] = (phase, f, O.solve_basic(phase, LAME10, f, tol=1e-8))
    return _REF[key]


def shape_for(kind, n):
    """A small grid whose `kind` axis has n points (array order z, y, x)."""
    return {"x": (4, 6, n), "y": (4, n, 16), "outer": (n, 4, 16)}[kind]


@pytest.mark.parametrize("n", LONG)
@pytest.mark.parametrize("kind", ["x", "y", "outer"])
def test_every_variant_matches_the_oracle(torch_dev, kind, n):
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    shape = shape_for(kind, n)
    phase, f, ref = reference(shape, 40 + n)
    plan = Plan([shape], prec="f32")
    v0, nv = plan.schedule(kind, n)
    assert v0 == 0 and nv == 3, (kind, n, v0, nv)
    for v in range(nv):
        say(f"FP32 schedule variant {kind} {n} v{v} on {shape}")
        plan.set_schedule(kind, n, v)
        assert plan.schedule(kind, n)[0] == v
        out, rep = plan.solve(torch.from_numpy(phase).to(dev), LAME10, torch.from_numpy(f).to(dev).float(),
                              tol=1e-8)
        torch.cuda.synchronize()
        err = O.relative_strain_error_voigt(out["eps"].double().cpu().numpy(), O.to_voigt(ref.eps))
        print(f"variant {v}: status={rep.status} iters={rep.iters}/{ref.iters} residual={rep.residual:.2e} "
              f"err={err:.2e}")
        assert rep.status in (0, 1)
        assert err < 1e-5
    plan.close()


def test_schedule_argument_checks(torch_dev):
    from paper_2601_00822_amd import Plan, LsfftError
    say("schedule argument checks")
    plan = Plan([(16, 16, 16)], prec="f32")
    assert plan.schedule("outer", 16) == (0, 1)        # short lengths: the default only
    with pytest.raises(LsfftError):
        plan.set_schedule("outer", 16, 1)
    with pytest.raises(LsfftError):
        plan.set_schedule("outer", 256, 3)
    plan.close()
    p64 = Plan([(16, 16, 256)], prec="f64")
    assert p64.schedule("x", 256) == (0, 1)            # FP64: the default only
    assert p64.schedule("layout", 0) == (0, 2)         # FP64 plans start in rows
    table = p64.autotune(iters=2)                      # and tune the layout only
    assert sorted((e["kind"], e["len"], e["variant"]) for e in table) == [("layout", 0, 0), ("layout", 0, 1)]
    assert p64.schedule("layout", 0)[0] == [e["variant"] for e in table if e["chosen"]][0]
    p64.close()
    p2d = Plan([(16, 64)], prec="f32")
    assert p2d.autotune(iters=2) == []                 # 2D: nothing to tune
    p2d.close()


def test_autotune_choice_solves_like_the_oracle_and_is_cached(torch_dev, tmp_path):
    """The tuner times every variant of the 48^3 and 4x64x96 grids' passes,
    keeps the fastest per (kind, length), then times both spectral layouts
    of each grid and keeps the faster, writes them to the cache, and a plan
    built with LSFFT_TUNE_CACHE naming that file starts from the same
    choices; the tuned plan's solves match the oracle (FP32 bar) in a mixed
    batch."""
    torch, dev = torch_dev
    from paper_2601_00822_amd import Plan
    shapes = [(48, 48, 48), (4, 64, 96)]
    cache = tmp_path / "tune.json"
    say("autotune 48^3 + 4x64x96, 8 iterations per variant")
    plan = Plan(shapes, prec="f32", max_batch=2)
    table = plan.autotune(iters=8, cache_path=str(cache))
    for e in table:
        print(e)
    keys = {(e["kind"], e["len"]) for e in table if e["kind"] != "layout"}
    assert keys == {("x", 48), ("y", 48), ("outer", 48), ("x", 96), ("y", 64)}
    # one layout pair per grid (both have nx a multiple of 16)
    lay = {}
    for g in range(len(shapes)):
        rows = [e for e in table if e["kind"] == "layout" and e["len"] == g]
        assert sorted(e["variant"] for e in rows) == [0, 1] and all(e["us"] > 0 for e in rows)
        best = min(rows, key=lambda e: (e["us"], -e["variant"]))
        assert [e["variant"] for e in rows if e["chosen"]] == [best["variant"]]
        assert plan.schedule("layout", g)[0] == best["variant"]
        lay[g] = best["variant"]
    for k in keys:
        rows = [e for e in table if (e["kind"], e["len"]) == k]
        assert sorted(e["variant"] for e in rows) == list(range(plan.schedule(*k)[1]))
        best = min(rows, key=lambda e: e["us"])
        assert [e["variant"] for e in rows if e["chosen"]] == [best["variant"]]
        assert all(e["us"] > 0 for e in rows)
        assert plan.schedule(*k)[0] == best["variant"]
    cached = json.loads(cache.read_text())
    for kind, n in keys:
        assert cached[f"f32/3d/{kind}/{n}"] == plan.schedule(kind, n)[0]
    lkey = {g: "f32/3d/layout/%dx%dx%d" % shp[::-1] for g, shp in enumerate(shapes)}
    for g in lay:
        assert cached[lkey[g]] == lay[g]
    # the tuned plan solves like the oracle
    probs, refs = [], []
    for g, shp in enumerate(shapes):
        phase, f, ref = reference(shp, 70 + g)
        probs.append(dict(grid=g, phase=torch.from_numpy(phase).to(dev), lame=LAME10,
                          f=torch.from_numpy(f).to(dev).float()))
        refs.append(ref)
    outs, reps, st = plan.solve_batch(probs, tol=1e-8)
    for o, r, ref in zip(outs, reps, refs):
        err = O.relative_strain_error_voigt(o["eps"].double().cpu().numpy(), O.to_voigt(ref.eps))
        print(f"tuned: iters={r.iters} residual={r.residual:.2e} err={err:.2e}")
        assert r.status in (0, 1) and err < 1e-5
    plan.close()
    # a new plan reads the cache named by the environment
    os.environ["LSFFT_TUNE_CACHE"] = str(cache)
    try:
        p2 = Plan(shapes, prec="f32")
        for kind, n in keys:
            assert p2.schedule(kind, n)[0] == cached[f"f32/3d/{kind}/{n}"]
        for g in lay:
            assert p2.schedule("layout", g)[0] == lay[g]
        p2.close()
    finally:
        del os.environ["LSFFT_TUNE_CACHE"]
