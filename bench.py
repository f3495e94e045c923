"""Throughput benchmark of the BFCS Lippmann-Schwinger solver on one MI355X.

A step is one complete BFCS solve of the default workload, the largest
single-GPU configuration: 3D 256^3 voxels = 16^3 unit cells of 16^3, random
non-overlapping spheres (volume fraction 0.3, radii 3-6 voxels) in every
cell, stiff inclusions at Young's contrast 100, nu = 0.3, vector bump force
of radius 12 voxels with seeded centre and direction, reference medium = mean
of the extreme Lame constants, basic scheme, tol 1e-8, FP32 transforms and
updates under FP64 defect correction (the state, the residual and the
stopping test are FP64): force transform and free term, the iterations
until the FP64 residual meets the tolerance, and materialization of u, eps
and sigma.  Inputs are resident in HBM before the timed region starts.

Printed: one JSON line with voxel-iterations/s (sum of |N| x iterations over
the timed solves divided by wall time), solves/s, the roofline of the
dominant kernel (algorithmic bytes of its launches over their HIP-event
durations on a timed plan), the whole-solve bandwidth fraction, and the FP64
CPU oracle timed on a bounded sample of the same workload (one core, and
with its transforms on all cores).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxel-iters/s + BFCS solves/s at 1e-8 residual; surrogate vs solver speedup"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "bfcs128": dict(shape=(128, 128, 128), cell=16, vf=0.25, contrast=10.0, radius=12.0,
                    desc="3D 128^3 (8^3 cells of 16^3), one sphere per cell vf 0.25, contrast 10, "
                         "vector bump R=12, basic scheme to 1e-8"),
    "bfcs256": dict(shape=(256, 256, 256), cell=16, vf=0.30, contrast=100.0, radius=12.0, rsa=True,
                    desc="3D 256^3 (16^3 cells of 16^3), RSA spheres vf 0.3 r 3-6, stiff inclusions "
                         "contrast 100, vector bump R=12, to 1e-8"),
    "bfcs256soft": dict(shape=(256, 256, 256), cell=16, vf=0.30, contrast=0.01, radius=12.0, rsa=True,
                        desc="3D 256^3 (16^3 cells of 16^3), RSA spheres vf 0.3 r 3-6, soft inclusions "
                             "contrast 0.01, vector bump R=12, to 1e-8"),
    "surrogate": dict(surrogate=True, desc="learned surrogate: 64^3 grid, one sphere per 16^3 cell (vf 0.25, "
                                            "contrast 10); forces of 1-3 bumps R 4-12; targets = translation "
                                            "averages over all 4096 intra-cell shifts (FP64 solver kernel) "
                                            "restricted to 32^3; Fourier neural operator 4 layers, width 32, "
                                            "12 modes, bf16 MFMA training and inference"),
    "fno_step": dict(fno_step=True, desc="surrogate kernels alone: training steps and inference batches of the "
                                          "4-layer, width-32, 12-mode operator on 32^3 inputs (seeded random "
                                          "data, batch 32)"),
    "batch512": dict(batch=True, desc="512 solves in one call: 8 microstructures (48^3, 64^3, 96^3 "
                                      "round robin, cells of 16^3, RSA spheres r 3-6, vf U[0.10,0.35], "
                                      "contrast log-uniform [2,100]) x 64 seeded intra-cell shifts, "
                                      "bump R=8, translated averages accumulated in FP64"),
}


def precision_note(args) -> str:
    if args.prec == "f64":
        return "f64 throughout"
    if args.refine:
        return ("f32 transforms and updates in the inner solves; f64 state, residual, stopping test and "
                "averaging (defect correction); iterations counted = f32 inner iterations only")
    return "f32 transforms/updates and state, f64 residual sums and stopping test"


def make_batch(seed: int = 0):
    """Eight averaging groups of the batched workload (inputs only)."""
    import numpy as np
    import gen
    rng = np.random.default_rng(seed)
    sizes = [48, 64, 96, 48, 64, 96, 48, 64]
    groups = []
    for k, n in enumerate(sizes):
        shape = (n, n, n)
        vf = float(rng.uniform(0.10, 0.35))
        contrast = float(np.exp(rng.uniform(np.log(2.0), np.log(100.0))))
        cell, vf_got = gen.rsa_cell(16, 3, vf, 3.0, 6.0, seed=seed * 100 + k)
        phase = gen.tile_cell(cell, shape)
        f = gen.bump_force(shape, gen.random_center(shape, seed * 100 + k), 8.0,
                           gen.random_direction(3, seed * 100 + k + 50))
        shifts = gen.sample_shifts(16, 3, 64, seed * 100 + k)
        table = gen.Material.two_phase(1.0, contrast).table()
        groups.append(dict(shape=shape, phase=phase, f=f, table=table, shifts=shifts, vf=vf_got,
                           contrast=contrast))
    return groups


def run_batch_workload(args, wl):
    """Batched translated averaging: one lsfft_translate_average_batch call per step."""
    import numpy as np
    import torch
    from paper_2601_00822_amd import Plan, lame_from_young
    dev = torch.device("cuda:0")
    groups = make_batch(0)
    shapes = sorted({g["shape"] for g in groups})
    dt = torch.float32 if args.prec == "f32" else torch.float64
    dgroups = []
    for g in groups:
        dgroups.append(dict(grid=shapes.index(g["shape"]), phase=torch.from_numpy(g["phase"]).to(dev),
                            lame=lame_from_young(g["table"]), f=torch.from_numpy(g["f"]).to(dev).to(dt),
                            shifts=g["shifts"]))
    nsolve = sum(len(g["shifts"]) for g in groups)
    plan = Plan(shapes, prec=args.prec, scheme=args.scheme, max_batch=nsolve, refine=args.refine)
    tune = [] if args.no_autotune else plan.autotune(iters=20)
    for _ in range(args.warmup):
        plan.translate_average_batch(dgroups, tol=1e-8)
    torch.cuda.synchronize()
    vox_iters = 0
    iters_all = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, reps, st = plan.translate_average_batch(dgroups, tol=1e-8)
        k = 0
        for g in groups:
            nv = int(np.prod(g["shape"]))
            for _ in range(len(g["shifts"])):
                vox_iters += nv * reps[k].iters
                iters_all.append(reps[k].iters)
                k += 1
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # whole job: algorithmic bytes of every solver kernel per iteration of
    # each solve's grid times its iterations, over the wall time
    from paper_2601_00822_amd import K_GREEN, K_XPASS, K_YPASS, K_REDUCE, K_CGUPD
    classes = (K_GREEN, K_XPASS, K_YPASS, K_REDUCE, K_CGUPD)
    grid_of = [dg["grid"] for dg in dgroups for _ in range(len(dg["shifts"]))]
    bytes_iter = {g: sum(plan.iteration_bytes(k, g) for k in classes) for g in range(len(shapes))}
    job_bytes = args.steps * sum(bytes_iter[g] * r.iters for g, r in zip(grid_of, reps))
    plan.close()
    # kernel-duration region: one more batch on a timed plan (graphs off, a
    # HIP event pair stamped by every launch)
    plan_t = Plan(shapes, prec=args.prec, scheme=args.scheme, max_batch=nsolve, refine=args.refine, timing=True)
    for e in tune:
        if e["chosen"]:
            plan_t.set_schedule(e["kind"], e["len"], e["variant"])
    plan_t.translate_average_batch(dgroups, tol=1e-8)
    plan_t.kernel_times_reset()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, reps_t, _ = plan_t.translate_average_batch(dgroups, tol=1e-8)
    torch.cuda.synchronize()
    elapsed_t = time.perf_counter() - t1
    per, dom = class_rooflines(plan_t, [(g, r.iters) for g, r in zip(grid_of, reps_t)], args.scheme != "basic")
    plan_t.close()
    statuses = sorted({r.status for r in reps})
    return {
        "metric": METRIC, "value": vox_iters / elapsed, "unit": "voxel-iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": "batch512", "solves": nsolve, "grids": [list(s) for s in shapes],
                   "scheme": args.scheme, "description": wl["desc"], "precision": precision_note(args),
                   "contrasts": [round(g["contrast"], 2) for g in groups],
                   "volume_fractions": [round(g["vf"], 3) for g in groups]},
        "solves_per_s": nsolve * args.steps / elapsed,
        "iterations": {"min": int(min(iters_all)), "max": int(max(iters_all)),
                       "mean": float(np.mean(iters_all))},
        "statuses": statuses,
        "whole_job": {"gbs": job_bytes / elapsed / 1e9, "frac": job_bytes / elapsed / 1e9 / HBM_PEAK_GBS,
                      "note": "algorithmic bytes of all solver kernels per iteration of each solve's grid x its "
                              "iterations / wall time"},
        "kernel_gbs": {k: round(v["gbs"], 1) for k, v in per.items()},
        "timing_region": {"seconds": elapsed_t,
                          "note": "one batch with graphs off and a HIP event pair stamped at every kernel's start "
                                  "and end; kernel bandwidths and the roofline come from this region"},
        "roofline": roofline_field(per, dom, None),
        "autotune": {"schedule": {f"{e['kind']}/{e['len']}": e["variant"] for e in tune if e["chosen"]},
                     "us_per_launch": {f"{e['kind']}/{e['len']}/v{e['variant']}": round(e["us"], 2) for e in tune}},
    }


def run_surrogate_workload(args, wl):
    """Averaged-strain kernel from the FP64 solver, dataset, training,
    held-out error against the solver, the per-input fallback, and the
    surrogate's speedup over the solver and over the kernel convolution."""
    import numpy as np
    import torch
    import gen
    from paper_2601_00822_amd import Plan, lame_from_young, bump_forces, block_mean, sample_norms
    from paper_2601_00822_amd import surrogate as S
    from paper_2601_00822_amd.fno import FnoArch, Surrogate

    def log(msg):
        print(f"[surrogate] {msg}", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    n, cell = 64, 16
    phase_np, vf = gen.inclusion_per_cell((n, n, n), cell, 0.25)
    lame = lame_from_young(gen.Material.two_phase(1.0, 10.0).table())
    phase = torch.from_numpy(phase_np).to(dev)
    t0 = time.perf_counter()
    K, Ku, kreps = S.averaged_kernels(phase, lame, cell, prec="f64", max_batch=512)
    torch.cuda.synchronize()
    t_kernel = time.perf_counter() - t0
    log(f"averaged-strain kernel: {len(kreps)} FP64 solves in {t_kernel:.1f} s, "
        f"max residual {max(r.residual for r in kreps):.2e}")
    conv_plan = Plan([(n, n, n)], prec="f64", max_batch=64)

    def make(count, seed):
        params = gen.bump_set_params(n, count, seed)
        X, T = [], []
        for k in range(0, count, 64):
            f = bump_forces((n, n, n), params[k:k + 64], device=dev)
            e = S.averaged_strain_from_kernel(K, f, plan=conv_plan)
            X.append(S.restrict2(f, dtype=torch.float32))
            T.append(S.restrict2(e, dtype=torch.float32))
        return torch.cat(X).contiguous(), torch.cat(T).contiguous(), params

    t0 = time.perf_counter()
    Xtr, Ttr, _ = make(args.train_samples, 1)
    Xte, Tte, pte = make(args.test_samples, 2)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    # normalisation: root mean square of the training inputs and targets
    xs = float(np.sqrt(np.sum(sample_norms(Xtr)[1] ** 2) / Xtr.numel()))
    ts = float(np.sqrt(np.sum(sample_norms(Ttr)[1] ** 2) / Ttr.numel()))
    log(f"dataset: {Xtr.shape[0]} train / {Xte.shape[0]} held-out pairs in {t_data:.1f} s")
    arch = FnoArch()
    model = Surrogate(arch, max_batch=args.fno_batch)
    model.set_params(S.init_params(arch, 0))
    Xn = block_mean(Xtr, 1, scale=1.0 / xs)
    Tn = block_mean(Ttr, 1, scale=1.0 / ts)
    del Xtr, Ttr
    tr = S.train(model, Xn, Tn, epochs=args.epochs, batch=args.fno_batch, lr=args.lr,
                 seed=3, log_every=200, printer=log)
    del Xn, Tn
    log(f"training: {tr.steps} steps in {tr.seconds:.1f} s ({1e3 * tr.seconds / max(tr.steps, 1):.2f} ms/step)")
    Y = block_mean(S.predict(model, block_mean(Xte, 1, scale=1.0 / xs), args.fno_batch), 1, scale=ts)
    err = S.relative_l2(Y, Tte)
    log(f"held-out relative L2: mean {err.mean():.4f} max {err.max():.4f}")
    trained = S.TrainedSurrogate(model, xs, ts, float(err.mean()), float(err.max()))

    # the FP64 solver as judge: direct translation averages of held-out forces
    plan64 = Plan([(n, n, n)], prec="f64", max_batch=512)
    checks = []
    t_direct = 0.0
    for i in range(args.direct_checks):
        f = bump_forces((n, n, n), [pte[i]], device=dev)[0]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        avg, _ = plan64.translate_average(phase, lame, f, S.cell_shifts(cell), tol=1e-8)
        torch.cuda.synchronize()
        t_direct = time.perf_counter() - t1
        direct = S.restrict2(avg[6:12].contiguous(), dtype=torch.float32)
        checks.append({"surrogate_vs_direct": float(S.relative_l2(Y[i:i + 1], direct[None])[0]),
                       "kernel_target_vs_direct": float(S.relative_l2(Tte[i:i + 1], direct[None])[0])})
        log(f"direct FP64 check {i}: {checks[-1]} ({t_direct:.1f} s)")
    plan64.close()
    # solver time for one averaged field with the benchmark solver (FP32 + FP64 correction)
    plan32 = Plan([(n, n, n)], prec="f32", max_batch=512, refine=True)
    f = bump_forces((n, n, n), [pte[0]], device=dev, dtype=torch.float32)[0]
    plan32.translate_average(phase, lame, f, S.cell_shifts(cell)[:64], tol=1e-8)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan32.translate_average(phase, lame, f, S.cell_shifts(cell), tol=1e-8)
    torch.cuda.synchronize()
    t_solver = time.perf_counter() - t1
    plan32.close()
    # the kernel route: one convolution with the averaged kernel per field
    fb = bump_forces((n, n, n), pte[:args.fno_batch], device=dev)
    S.averaged_strain_from_kernel(K, fb, plan=conv_plan)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    S.averaged_strain_from_kernel(K, fb, plan=conv_plan)
    torch.cuda.synchronize()
    t_conv = (time.perf_counter() - t1) / fb.shape[0]
    # surrogate inference time per averaged field (batched)
    xb = block_mean(Xte[:args.fno_batch], 1, scale=1.0 / xs)
    model.forward(xb)
    torch.cuda.synchronize()
    reps = 20
    t1 = time.perf_counter()
    for _ in range(reps):
        model.forward(xb)
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t1) / (reps * xb.shape[0])
    # serving with the per-input judge: every held-out force, 2 % bound
    served, src = S.averaged_strain(bump_forces((n, n, n), pte[:args.fno_batch], device=dev), 0.02, trained,
                                    phase, lame, cell, kernel=K)
    served_err = S.relative_l2(served, Tte[:args.fno_batch])
    nonlocal_leg = run_nonlocal_leg(Ku, n, conv_plan, args, log, lame=lame, vf=vf)
    conv_plan.close()
    speedup = t_solver / t_inf
    log(f"solver {t_solver:.2f} s, kernel convolution {1e6 * t_conv:.1f} us, surrogate {1e6 * t_inf:.1f} us "
        f"per field")
    model.close()
    return {
        "metric": METRIC, "value": speedup, "unit": "x (solver s / surrogate s per averaged field)",
        "n_gpus": 1, "steps": tr.steps, "warmup": 0, "ms_per_step": 1e3 * tr.seconds / max(tr.steps, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "surrogate", "description": wl["desc"], "grid": [n, n, n], "coarse": [32, 32, 32],
                   "train_samples": args.train_samples, "heldout_samples": int(Xte.shape[0]),
                   "epochs": args.epochs, "batch": args.fno_batch, "lr": args.lr,
                   "arch": {"layers": arch.layers, "width": arch.width, "modes": arch.modes,
                            "hidden": arch.hidden}},
        "heldout_rel_l2": {"mean": float(err.mean()), "median": float(np.median(err)),
                           "p95": float(np.quantile(err, 0.95)), "p99": float(np.quantile(err, 0.99)),
                           "max": float(err.max()), "above_2pct": int(np.sum(err > 0.02))},
        "served_with_per_input_judge": {"batch": int(served.shape[0]), "from_surrogate": src.count("surrogate"),
                                        "from_kernel": src.count("kernel"),
                                        "max_rel_l2": float(np.max(served_err))},
        "speedup_vs_kernel_convolution": t_conv / t_inf,
        "direct_fp64_checks": checks,
        "nonlocal_operator": nonlocal_leg,
        "final_train_loss": float(np.mean(tr.losses[-50:])),
        "seconds": {"kernel_solves": t_kernel, "dataset": t_data, "training": tr.seconds,
                    "solver_per_field_f32": t_solver, "solver_per_field_f64": t_direct,
                    "kernel_convolution_per_field": t_conv, "surrogate_per_field": t_inf},
    }


def run_nonlocal_leg(Ku, n, conv_plan, args, log, lame=None, vf=None):
    """The nonlocal kernel surrogate (Eqs. 6.5-6.6, displacement type) on
    the same microstructure: pairs (<u>_k, -b_k) from the averaged
    displacement kernel, normal equations on the device, closed-form and
    Adam fits per kernel form and horizon, held-out relative residuals
    against the force and against its equilibrated part."""
    import numpy as np
    import torch
    import gen
    from paper_2601_00822_amd import bump_forces
    from paper_2601_00822_amd import nonlocal_operator as NL
    dev = Ku.device
    M = 6
    fits = [(0, 3.0), (0, 5.0), (0, 7.0), (1, 3.0), (1, 5.0)]     # (form, horizon); form 1 in 3D up to 5
    ntr, nte = min(args.train_samples, 1024), min(args.test_samples, 256)
    nes = {k: NL.NormalEquations(M, k[1], form=k[0]) for k in fits}
    t_ne = {k: 0.0 for k in fits}
    ptr = gen.bump_set_params(n, ntr, 11)
    for k0 in range(0, ntr, 64):
        u, gam = NL.pairs(Ku, bump_forces((n, n, n), ptr[k0:k0 + 64], device=dev), plan=conv_plan)
        for k in fits:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            nes[k].add(u, gam)
            t_ne[k] += time.perf_counter() - t1
    pte = gen.bump_set_params(n, nte, 12)
    tests = [NL.pairs(Ku, bump_forces((n, n, n), pte[k0:k0 + 64], device=dev), plan=conv_plan)
             for k0 in range(0, nte, 64)]
    out = {"degree": M, "train_pairs": ntr, "heldout_pairs": nte, "grid": [n, n, n], "fits": {}}
    for k in fits:
        form, dl = k
        ne = nes[k]
        s = float(np.trace(ne.G)) / len(ne.g)
        lam = 1e-10 * s
        ops = {"closed": NL.fit(ne, lam), "adam": NL.fit(ne, lam, adam_steps=20000, lr=1e-3)}
        row = {"seconds_per_pair_normal_equations": t_ne[k] / ntr}
        for name, op in ops.items():
            res = np.concatenate([op.relative_residual(u, g) for u, g in tests])
            req = np.concatenate([op.relative_residual(u, g, equilibrated=True) for u, g in tests])
            row[name] = {"c": [float(v) for v in op.c], "train_loss_rel": ne.loss(op.c, lam) / ne.gg,
                         "heldout_rel_residual": {"mean": float(res.mean()), "max": float(res.max())},
                         "heldout_rel_residual_equilibrated": {"mean": float(req.mean()), "max": float(req.max())}}
        u0 = tests[0][0]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ops["closed"].apply(u0)
        torch.cuda.synchronize()
        row["seconds_per_field_apply"] = (time.perf_counter() - t1) / u0.shape[0]
        if form == 1:
            C11, C12, C44 = ops["closed"].long_wave_stiffness()
            row["long_wave_stiffness"] = {"C11": C11, "C12": C12, "C44": C44, "bulk": (C11 + 2.0 * C12) / 3.0,
                                          "shear_44": C44, "shear_11_12": 0.5 * (C11 - C12)}
        key = f"{'matrix' if form else 'scalar'}/{dl}"
        out["fits"][key] = row
        log(f"nonlocal {key}: held-out relative residual closed {row['closed']['heldout_rel_residual']['mean']:.4f} "
            f"(equilibrated {row['closed']['heldout_rel_residual_equilibrated']['mean']:.4f}, max "
            f"{row['closed']['heldout_rel_residual_equilibrated']['max']:.4f}), adam "
            f"{row['adam']['heldout_rel_residual_equilibrated']['mean']:.4f}")
    if lame is not None and vf is not None:
        # Voigt and Reuss bounds of the two phases at the voxelized volume
        # fraction (matrix phase 0, inclusions phase 1)
        lam_p, mu_p = np.asarray(lame)[:, 0], np.asarray(lame)[:, 1]
        kap_p = lam_p + 2.0 * mu_p / 3.0
        fr = np.array([1.0 - vf, vf])
        out["phase_bounds"] = {"volume_fraction": float(vf),
                               "bulk": [float(1.0 / np.sum(fr / kap_p)), float(np.sum(fr * kap_p))],
                               "shear": [float(1.0 / np.sum(fr / mu_p)), float(np.sum(fr * mu_p))],
                               "note": "[Reuss, Voigt] of the phases' bulk and shear moduli"}
    return out


def run_fno_step_workload(args, wl):
    """Time the surrogate's training step and batched inference on seeded
    random data (the kernels alone, no dataset construction)."""
    import numpy as np
    import torch
    from paper_2601_00822_amd import surrogate as S
    from paper_2601_00822_amd.fno import FnoArch, Surrogate
    arch = FnoArch()
    B = args.fno_batch
    model = Surrogate(arch, max_batch=B)
    model.set_params(S.init_params(arch, 0))
    rng = np.random.default_rng(0)
    x = torch.from_numpy(rng.normal(size=(B, arch.cin) + (arch.n,) * 3).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.normal(size=(B, arch.cout) + (arch.n,) * 3).astype(np.float32)).cuda()
    for _ in range(args.warmup):
        model.train_step(x, t, 1e-4)
        model.forward(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        model.train_step(x, t, 1e-4)
    torch.cuda.synchronize()
    t_train = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        model.forward(x)
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t0) / args.steps
    model.close()
    return {
        "metric": METRIC, "value": B / t_inf, "unit": "surrogate fields/s (inference)", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t_train, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "fno_step", "description": wl["desc"], "batch": B},
        "train_ms_per_step": 1e3 * t_train, "inference_ms_per_batch": 1e3 * t_inf,
    }


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("kernels_impl.hpp", "fft_core.hpp"):
        with open(os.path.join(ROOT, "paper_2601_00822_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str, prec: str, variant: int = 0, layout: str = "blocked"):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel sources, on the schedule variant the
    timed run uses for that pass (every counter pass of the summary names
    its kernel, whose last template argument is the variant) and on the same
    spectral layout ("rows" or "blocked"); else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{prec}_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"kernel_source_hash:\s*(\w+)", text)
    m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_source_hash():
        return None
    line = next((ln for ln in text.splitlines() if ln.startswith("Kernel:")), "")
    measured = {int(v) for v in re.findall(r"k_%s<[^>]*?(\d+)>" % kernel, line)}
    if measured != {int(variant)}:
        return None
    m_lay = re.search(r"spectral_layout:\s*(\w+)", text)
    if not m_lay or m_lay.group(1) != layout:
        return None
    return float(m_bytes.group(1))


def make_inputs(wl: dict, seed: int = 0):
    import numpy as np
    import gen
    shape = wl["shape"]
    if wl.get("rsa"):
        cell, _ = gen.rsa_cell(wl["cell"], 3, wl["vf"], 3.0, 6.0, seed=seed)
        phase = gen.tile_cell(cell, shape)
    else:
        phase, _ = gen.inclusion_per_cell(shape, wl["cell"], wl["vf"])
    f = gen.bump_force(shape, gen.random_center(shape, seed), wl["radius"], gen.random_direction(3, seed + 1))
    table = gen.Material.two_phase(1.0, wl["contrast"]).table()
    return phase, f, table, np.asarray(table)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Threads this process may use: the machine's CPU share if the environment
    states it, else the affinity mask."""
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return min(int(env), aff)
    return aff


def _oracle_iteration_rate(phase, lame, f):
    """Time Algorithm 1 of the oracle on the full grid twice: stopped after
    the free term and the first residual (max_iter = 0), and after one more
    iteration (max_iter = 1).  The difference is the cost of one iteration.
    Returns (seconds per iteration, seconds of the longer run)."""
    from oracle import lsfft_oracle as O
    t0 = time.perf_counter()
    O.solve_basic(phase, lame, f, tol=1e-30, max_iter=0)
    ta = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.solve_basic(phase, lame, f, tol=1e-30, max_iter=1)
    tb = time.perf_counter() - t0
    return max(tb - ta, 1e-6), tb


def cpu_baseline(wl: dict, phase, f, table):
    """The FP64 oracle as it stands, timed on the host on a bounded sample of
    the same workload: one iteration of Algorithm 1 on the full grid (the
    time of a run stopped after one iteration minus that of a run stopped
    before it).  First with its transforms as written (numpy.fft, one
    thread); then the same code with its two transform helpers routed to
    scipy.fft on all the host threads (the pointwise NumPy work stays
    single-threaded)."""
    from oracle import lsfft_oracle as O
    lame = O.lame_from_young(table)
    nvox = int(phase.size)
    per1, run1 = _oracle_iteration_rate(phase, lame, f)
    out = {"value": nvox / per1, "unit": "voxel-iters/s", "cores": 1, "kind": "oracle",
           "sample": f"one iteration of Algorithm 1 on the full {phase.shape} grid in FP64 NumPy (numpy.fft, "
                     f"single thread): {per1:.1f} s, the difference of runs stopped after and before it "
                     f"(the longer {run1:.1f} s)",
           "cpu_model": cpu_model(), "host_threads": host_threads()}
    try:
        import scipy.fft as sfft
    except ImportError:
        return out
    workers = host_threads()
    keep = (O.fft_r, O.ifft_r)

    def fft_r(a, shape):
        lead = a.ndim - len(shape)
        return sfft.rfftn(a, axes=tuple(range(lead, a.ndim)), workers=workers)

    def ifft_r(a, shape):
        lead = a.ndim - len(shape)
        return sfft.irfftn(a, s=shape, axes=tuple(range(lead, a.ndim)), workers=workers)

    O.fft_r, O.ifft_r = fft_r, ifft_r
    try:
        pern, _ = _oracle_iteration_rate(phase, lame, f)
    finally:
        O.fft_r, O.ifft_r = keep
    out["all_cores"] = {"value": nvox / pern, "unit": "voxel-iters/s", "cores": workers,
                        "sample": f"the same oracle code with its transforms by scipy.fft(workers={workers}): "
                                  f"{pern:.1f} s per iteration"}
    return out


CLASS_NAMES = ("green", "xpass", "ypass", "reduce", "cgupd")


def class_rooflines(plan_t, solves, two_outer: bool):
    """Per kernel class of a timed plan: total HIP-event time, launches,
    algorithmic bytes and bandwidth.  ``solves`` lists (grid index,
    iterations) of every solve the timed region ran; a class's algorithmic
    bytes are the sum over those solves of its bytes per iteration
    (lsfft_iteration_bytes) times the iterations.  Launches past a solve's
    convergence inside a polling round are gated and nearly empty; their
    time stays in the total.  Returns (per-class dict, dominant class): the
    dominant class is the one kernel with the most time (the y-pass class
    holds two kernels per iteration, the inverse and the forward sweep; the
    CG outer-pass class two, A p and the new direction)."""
    from paper_2601_00822_amd import K_GREEN, K_XPASS, K_YPASS, K_REDUCE, K_CGUPD
    ids = {"green": K_GREEN, "xpass": K_XPASS, "ypass": K_YPASS, "reduce": K_REDUCE, "cgupd": K_CGUPD}
    kernels_per_iter = {"green": 2.0 if two_outer else 1.0, "xpass": 1.0, "ypass": 2.0, "reduce": 1.0,
                        "cgupd": 1.0}
    out = {}
    iters_total = sum(it for _, it in solves)
    for name in CLASS_NAMES:
        ms, launches = plan_t.kernel_times(ids[name])
        if launches == 0:
            continue
        byts = sum(plan_t.iteration_bytes(ids[name], g) * it for g, it in solves)
        out[name] = {"ms": ms, "launches": launches, "bytes": byts,
                     "gbs": byts / (ms / 1e3) / 1e9 if ms > 0 else 0.0,
                     "kernels_per_iter": kernels_per_iter[name], "iterations": iters_total}
    cands = [k for k in ("green", "xpass", "ypass") if k in out]
    dom = max(cands, key=lambda k: out[k]["ms"] / out[k]["kernels_per_iter"])
    return out, dom


def roofline_field(per, dom, traffic):
    d = per[dom]
    kpi = d["kernels_per_iter"]
    working = d["iterations"] * kpi
    # one launch of the dominant kernel per iteration of each solve in a
    # single solve; in a batch one launch covers every running solve, so the
    # per-launch figures there are per solve-iteration
    bytes_per_launch = d["bytes"] / max(working, 1)
    per_launch_s = d["ms"] / 1e3 / max(working, 1)
    achieved = d["gbs"]
    return {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "algorithmic_bytes_per_launch": bytes_per_launch, "mean_launch_us": per_launch_s * 1e6,
            "launches": d["launches"], "working_launches": int(working)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="bfcs256", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default="f32", choices=["f32", "f64"])
    ap.add_argument("--scheme", default="basic", choices=["basic", "cg", "cg_plain", "anderson"])
    ap.add_argument("--no-refine", action="store_true",
                    help="FP32 without the FP64 defect correction (stops at the FP32 stagnation floor)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default schedule of every pass instead of autotuning it")
    ap.add_argument("--train-samples", type=int, default=20000)
    ap.add_argument("--test-samples", type=int, default=512)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--fno-batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--direct-checks", type=int, default=2)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before the solves, run one plain device-to-device copy of this many MiB "
                         "(reference dispatch for HBM byte counters)")
    args = ap.parse_args()
    args.refine = args.prec == "f32" and not args.no_refine
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the solver path is single-GPU (requested --gpus {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        return 2
    import numpy as np
    import torch
    from paper_2601_00822_amd import Plan, K_GREEN, K_XPASS, K_YPASS, K_REDUCE, K_CGUPD

    wl = WORKLOADS[args.workload]
    if wl.get("batch"):
        print(json.dumps(run_batch_workload(args, wl)))
        return 0
    if wl.get("surrogate"):
        print(json.dumps(run_surrogate_workload(args, wl)))
        return 0
    if wl.get("fno_step"):
        print(json.dumps(run_fno_step_workload(args, wl)))
        return 0
    dev = torch.device("cuda:0")
    phase, f, table, _ = make_inputs(wl)
    from paper_2601_00822_amd import lame_from_young
    lame = lame_from_young(table)
    dt = torch.float32 if args.prec == "f32" else torch.float64
    phase_d = torch.from_numpy(phase).to(dev)
    f_d = torch.from_numpy(f).to(dev).to(dt)
    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # timed region: iterations replayed as captured HIP graphs
    plan = Plan([wl["shape"]], prec=args.prec, scheme=args.scheme, refine=args.refine)
    # the library's autotuner picks each pass's schedule for this grid (before
    # the timed region); the kernel-duration plan starts from the same choice
    tune, tune_s = [], 0.0
    if not args.no_autotune:
        t0 = time.perf_counter()
        tune = plan.autotune(iters=20)
        tune_s = time.perf_counter() - t0
    # kernel-duration region: the same solves with graphs off and a HIP
    # event pair stamped by every launch at its kernel's start and end
    plan_t = Plan([wl["shape"]], prec=args.prec, scheme=args.scheme, timing=True, refine=args.refine)
    for e in tune:
        if e["chosen"]:
            plan_t.set_schedule(e["kind"], e["len"], e["variant"])
    nvox = int(np.prod(wl["shape"]))

    for _ in range(args.warmup):
        plan.solve(phase_d, lame, f_d, tol=1e-8)
    plan_t.solve(phase_d, lame, f_d, tol=1e-8)
    torch.cuda.synchronize()
    iters = 0
    reps = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, rep = plan.solve(phase_d, lame, f_d, tol=1e-8)
        iters += rep.iters
        reps.append(rep)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    plan_t.kernel_times_reset()
    iters_t = 0
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # the kernel-duration region repeats at most three solves: each holds
    # hundreds to thousands of launches of every kernel
    steps_t = min(args.steps, 3)
    for _ in range(steps_t):
        _, rep = plan_t.solve(phase_d, lame, f_d, tol=1e-8)
        iters_t += rep.iters
    torch.cuda.synchronize()
    elapsed_t = time.perf_counter() - t1

    per, dom = class_rooflines(plan_t, [(0, iters_t)], args.scheme != "basic")
    # the counter summary counts only if it measured the variant this run
    # uses for the dominant pass (the default where nothing was tuned)
    kind = {"green": "outer", "xpass": "x", "ypass": "y"}.get(dom)
    traffic = None
    if kind is not None and len(wl["shape"]) == 3:
        axis = {"outer": wl["shape"][0], "y": wl["shape"][1], "x": wl["shape"][2]}[kind]
        layout = "blocked" if plan_t.schedule("layout", 0)[0] == 1 else "rows"
        traffic = measured_traffic(dom, args.workload, args.prec, plan_t.schedule(kind, axis)[0], layout)
    # whole solve: algorithmic bytes of every solver kernel per iteration
    # times the iterations, over the wall time of the graph region (host
    # polls, setup, FP64 correction and materialization included)
    bytes_iter = sum(plan.iteration_bytes(k) for k in (K_GREEN, K_XPASS, K_YPASS, K_REDUCE, K_CGUPD))
    solve_gbs = bytes_iter * iters / elapsed / 1e9

    out = {
        "metric": METRIC,
        "value": nvox * iters / elapsed,
        "unit": "voxel-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": list(wl["shape"]), "scheme": args.scheme,
                   "precision": precision_note(args), "tol": 1e-8,
                   "description": wl["desc"]},
        "solves_per_s": args.steps / elapsed,
        "iterations_per_solve": iters / args.steps,
        "final_residual": reps[-1].residual,
        "status": reps[-1].status,
        "kernel_ms_per_iteration": {k: v["ms"] / max(iters_t, 1) for k, v in per.items()},
        "kernel_gbs": {k: round(v["gbs"], 1) for k, v in per.items()},
        "whole_solve": {"gbs": solve_gbs, "frac": solve_gbs / HBM_PEAK_GBS,
                        "bytes_per_iteration": bytes_iter,
                        "note": "algorithmic bytes of all solver kernels per iteration x iterations / wall time "
                                "of the timed region"},
        "timing_region": {"value": nvox * iters_t / elapsed_t, "solves": steps_t,
                          "note": "same solves with graphs off and a HIP event pair stamped at every kernel's "
                                  "start and end (hipExtLaunchKernelGGL); kernel durations and the roofline come "
                                  "from this region"},
        "roofline": roofline_field(per, dom, traffic),
        "autotune": {"seconds": tune_s,
                     "schedule": {f"{e['kind']}/{e['len']}": e["variant"] for e in tune if e["chosen"]},
                     "us_per_launch": {f"{e['kind']}/{e['len']}/v{e['variant']}": round(e["us"], 2) for e in tune}},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, phase, f, table)
    plan.close()
    plan_t.close()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
