#!/usr/bin/env python3
"""Throughput of the lifted-PROPELLER hot path on one MI355X.

A step is one optimiser update of the whole hot path over one synthetic slice:
sheared spectral projection of every blade, forward 2D DFT, mask and residual,
inverse 2D DFT, transposed-shear gather with the TV gradient and the Adam update.
Every step counts one forward+adjoint per blade, so the reported value is
blade forward+adjoint evaluations per second.

Timed region: K steps replayed from a captured HIP graph, inputs resident in HBM,
bracketed by device synchronisation. Stage durations come from HIP events recorded
on the session's own stream around every stage over K further (eager) steps.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP32_VALU_TFLOPS = 78.6      # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz, no packed FP32
METRIC = "blade fwd+adjoint/s and recon wall-time vs plain loop; served p50/p99 latency"
_T0 = time.perf_counter()


def progress(msg: str) -> None:
    """A progress line on stderr (the JSON result is the only line on stdout)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def parse_args(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="dynamic_192", choices=["static_64", "static_256", "dynamic_192"])
    ap.add_argument("--tiles", default=None,
                    help="tile shape of the headline workload, comma-separated vp_tiles fields, instead of "
                         "autotuning (e.g. to profile one variant in several passes)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="approximate CPU oracle time budget")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain-loop leg")
    ap.add_argument("--no-kplanes", action="store_true", help="skip the K-Planes dynamic model leg")
    ap.add_argument("--no-static", action="store_true", help="skip the static 256^2 leg (when not the headline)")
    ap.add_argument("--no-nu", action="store_true", help="skip the blade-aligned sampling fit leg")
    ap.add_argument("--no-shard", action="store_true", help="skip the one-GPU share of a spectral split")
    ap.add_argument("--batch-slices", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--no-serve", action="store_true", help="skip the served-stream leg")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-steps", type=int, nargs=2, default=[40, 160], metavar=("STATIC", "DYNAMIC"))
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of known size (counter calibration)")
    return ap.parse_args(argv)


# ------------------------------------------------------------------ workload

def algorithmic(case):
    """Bytes and flops the method must move/do per step, per stage (static or dynamic)."""
    n, S, T, B = case.n, case.n_spec, case.n_time, case.n_blades
    vox = T * S * n * n
    px = B * n * n
    if T > 1:
        import numpy as np

        u = case.blade_times_or_zero() * (T - 1)
        k = np.minimum(np.floor(u), T - 2)
        a = u - k
        parts = int(np.sum((1.0 - a) != 0.0) + np.sum(a != 0.0))
    else:
        parts = B
    c8 = 8
    stage_bytes = {
        "project": vox * c8 + parts * n * n * c8,
        "rows_fwd": parts * n * n * c8 + px * c8,
        "cols": px * (c8 + c8 + c8 + 1),
        "rows_inv": 2 * px * c8,
        "gather_update": px * c8 + 48 * vox,
    }
    taps_flops = 16 * S * n * n * parts      # 4 bilinear taps x complex x FMA per voxel-part
    stage_flops = {
        "project": taps_flops,
        "gather_update": taps_flops + 60 * vox,
    }
    return stage_bytes, stage_flops, parts


def gpu_measurements(case, plan, B):
    """y_b = M_b (DFT2(P_b V_GT(tau_b)) + sigma n_b) with the HIP forward model."""
    import numpy as np
    import torch

    from synth.phantom import ground_truth_volume

    S = case.n_spec
    if case.n_time == 1:
        w, f = case.layers_at(0.0)
        gt = torch.from_numpy(ground_truth_volume(w, f, S)[None].astype(np.complex64)).cuda()
        k = B.vp_forward(plan, gt).cpu().numpy()
    else:
        k = np.zeros((case.n_blades, case.n, case.n), dtype=np.complex64)
        for b in range(case.n_blades):
            pb = B.Plan(case.n, S, 1, case.angle_rad[b:b + 1], case.lines[b:b + 1], None, case.spec_shift_px)
            w, f = case.layers_at(float(case.blade_time[b]))
            gt = torch.from_numpy(ground_truth_volume(w, f, S)[None].astype(np.complex64)).cuda()
            k[b] = B.vp_forward(pb, gt).cpu().numpy()[0]
    mask = plan.masks()
    return (k + case.sigma * mask * case.noise).astype(np.complex64)


# ------------------------------------------------------------------ legs

def cpu_baseline(case, budget_s):
    """The FP64 oracle on the host: whole steps of the same workload, bounded in time."""
    import numpy as np

    import oracle as O

    geom = O.Geometry.from_dict(case.geometry())
    y = O.simulate_measurements(case)
    kw = dict(tv_weight=case.tv_weight, tv_eps=case.tv_eps, lr=case.lr)
    t0 = time.perf_counter()
    O.reconstruct(geom, y, 1, **kw)
    t1 = time.perf_counter() - t0
    k = int(max(1, min(50, math.floor(budget_s / max(t1, 1e-6)))))
    t0 = time.perf_counter()
    O.reconstruct(geom, y, k, **kw)
    el = time.perf_counter() - t0
    threads = 1  # NumPy FFT and elementwise kernels run on one thread
    return {"value": case.n_blades * k / el, "unit": "blades/s", "cores": threads, "kind": "oracle",
            "sample": f"{k} full optimiser steps of {case.name} (each {case.n_blades} blade fwd+adj, "
                      f"TV, Adam) plus one objective evaluation, FP64 NumPy, {el:.1f} s"}


def _slice_problem(case, B):
    plan = B.Plan.from_geometry(case.geometry())
    y = gpu_measurements(case, plan, B)
    return plan, y


def _warm_plans(probs, B):
    """Puts every plan's device tables and launch lists on the device (one forward each),
    so that no timed pass pays a plan's one-time set-up that the passes after it reuse."""
    import torch

    for plan, _ in probs:
        B.vp_forward(plan, torch.zeros(plan.volume_shape, dtype=torch.complex64, device="cuda"))
    torch.cuda.synchronize()


def batched_leg(B, n_slices, steps, timed_steps=50):
    """64 independent slices: one-slice-at-a-time loop vs one batched, graph-captured run."""
    import numpy as np
    import torch

    from synth import configs

    cases = [configs.batch_slice(j) for j in range(n_slices)]
    probs = [_slice_problem(c, B) for c in cases]
    opts = [B.vp_options_default(n_steps=steps, tv_weight=c.tv_weight, lr=c.lr) for c in cases]
    # the batch takes one tile shape, tuned on its largest slice inside the timed call
    bopts = [B.vp_options_default(n_steps=steps, tv_weight=c.tv_weight, lr=c.lr, autotune=1) for c in cases]
    # warm both paths (every slice's tables uploaded, kernels loaded)
    B.vp_reconstruct(probs[0][0], probs[0][1], B.vp_options_default(n_steps=2))
    _warm_plans(probs, B)
    t0 = time.perf_counter()
    solo = [B.vp_reconstruct(p, y, o) for (p, y), o in zip(probs, opts)]
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    batch = B.vp_batch_reconstruct([p for p, _ in probs], [y for _, y in probs], bopts)
    t_batch = time.perf_counter() - t0
    same = all(np.array_equal(a["vol"], b["vol"]) for a, b in zip(solo, batch))
    blades = sum(c.n_blades for c in cases) * steps
    voxels = sum(c.n_spec * c.n * c.n for c in cases)
    step = batched_step(B, cases, probs, timed_steps)
    return {"workload": f"{n_slices} static slices, n in {{128,192,256}}, S in {{16,32}}, 8-16 blades, "
                        f"{steps} Adam steps each (seeds 4000+j)",
            "voxels": voxels, "plain_loop_s": round(t_plain, 4), "batched_s": round(t_batch, 4),
            "speedup_vs_plain_loop": round(t_plain / t_batch, 3),
            "blades_per_s_batched": round(blades / t_batch, 1), "blades_per_s_plain_loop": round(blades / t_plain, 1),
            "batched_equals_solo_bitwise": bool(same),
            "wall_times": "whole calls: upload, the batch's autotuning, graph capture, the steps, the objective "
                          "and the read-back (plain loop: the same per slice)",
            "step": step,
            "tiles": "batch: autotuned on its largest slice; plain loop: each plan's built-in shape"}


def batched_step(B, cases, probs, steps):
    """The batched step alone, steady state: the 64 slices resident (vp_batch), one captured
    step replayed `steps` times between device synchronisations (no upload, tuning, capture,
    objective or read-back inside), then per-stage HIP events over eager steps; the roofline
    of the dominant stage from the algorithmic bytes of all slices' work items."""
    import torch

    opts = [B.vp_options_default(n_steps=1 << 30, tv_weight=c.tv_weight, lr=c.lr, autotune=1) for c in cases]
    batch = B.Batch([p for p, _ in probs], [y for _, y in probs], opts)
    batch.step(5, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(steps, use_graph=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    stages = batch.stage_times(max(5, steps // 4))
    batch.close()
    tot = {}
    for c in cases:
        sb, _, _ = algorithmic(c)
        for k, v in sb.items():
            tot[k] = tot.get(k, 0) + v
    dom = max(stages, key=lambda k: stages[k])
    ach = tot[dom] / (stages[dom] * 1e-3) / 1e9
    blades = sum(c.n_blades for c in cases)
    return {"ms_per_step": round(el * 1e3 / steps, 5), "steps": steps,
            "blades_per_s": round(blades * steps / el, 1),
            "stage_ms": {k: round(v, 5) for k, v in stages.items()},
            "step_hbm_bytes_algorithmic": int(sum(tot.values())),
            "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                         "kernel": "k_gather<1>" if dom == "gather_update" else dom,
                         "kernel_ms": round(stages[dom], 5), "algorithmic_bytes_per_launch": tot[dom],
                         "note": "one launch per stage over every slice's work items; stage durations are "
                                 "HIP events on the batch's stream around each launch"}}


KP_MODEL = dict(features=8, tv_weight=1e-1, smooth_weight=1e-2, sparse_weight=1e-3, eps=1e-3)


def kplanes_leg(B, steps, warmup):
    """The K-Planes dynamic model (Section 4.1: six grids of 8 complex features, two scales
    at the image and half resolution, time nodes = the dense model's knots) fitted to the
    dynamic 192^2 workload: step throughput, per-kernel stage times, the roofline of the
    dominant kernel (vector ALU: a product of six factors per voxel, blade and feature) and
    the PSNR of the fitted video."""
    import numpy as np
    import torch

    from synth import configs
    from synth.kplanes_init import init_params

    case = configs.dynamic_192()
    plan = B.Plan.from_geometry(case.geometry())
    y = gpu_measurements(case, plan, B)
    res = (case.n, case.n // 2)
    model = B.vp_kplanes.make(KP_MODEL["features"], case.n_time, res, KP_MODEL["tv_weight"],
                              KP_MODEL["smooth_weight"], KP_MODEL["sparse_weight"], KP_MODEL["eps"])
    init = init_params(case.n_spec, KP_MODEL["features"], case.n_time, res, seed=case.seed)
    # the blade kernels of the per-blade plan take the autotuned tile shape
    opts = B.vp_options_default(n_steps=case.n_steps, lr=case.lr, device=0, autotune=1)
    sess = B.KPlanesSession(plan, model, y, init, opts)
    sess.step(warmup, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sess.step(steps, use_graph=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    stages = sess.stage_times(max(3, steps // 4))
    sess.close()
    # flops per launch of the heavy kernels: one complex product and one complex
    # multiply-add (14 flops) per voxel, blade, scale and feature
    vb = case.n_blades * case.n_spec * case.n * case.n
    fl = 14 * KP_MODEL["features"] * len(res) * vb
    heavy = {k: v for k, v in stages.items() if k in ("grad_z", "grad_x", "grad_y")}
    dom = max(heavy, key=lambda k: heavy[k])
    ach = fl / (heavy[dom] * 1e-3) / 1e12
    # quality: a whole fit, frames at the blade times against the phantom there
    r = B.vp_kplanes_reconstruct(plan, model, y, init, opts, frame_times=case.blade_time)
    truth = np.stack([sum(case.layers_at(float(t))) for t in case.blade_time]).astype(np.complex64)
    p_fit = B.vp_psnr(torch.from_numpy(r["proj"]).cuda(), torch.from_numpy(truth).cuda())[0].cpu().numpy()
    return {"workload": f"dynamic_192 geometry; K-Planes F {KP_MODEL['features']}, time nodes {case.n_time}, "
                        f"scales {res[0]} and {res[1]}",
            "value": round(case.n_blades * steps / el, 1), "unit": "blade fwd+adjoint/s",
            "ms_per_step": round(el * 1e3 / steps, 5), "steps": steps,
            "stage_ms": {k: round(v, 5) for k, v in stages.items()},
            "roofline": {"bound": "alu", "achieved": round(ach, 3), "peak": FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(ach / FP32_VALU_TFLOPS, 4), "traffic": None, "kernel": f"k_kp_{dom}",
                         "kernel_ms": round(heavy[dom], 5), "algorithmic_flops_per_launch": fl},
            "quality": {"psnr_db": round(float(np.mean(p_fit)), 2), "frames": int(len(case.blade_time)),
                        "steps": case.n_steps, "model": KP_MODEL}}


def gpu_samples(case, plan, B):
    """Blade-aligned samples y_b = A_b(P_b V_GT(tau_b)) + sigma n_b[:L_b] with the HIP
    gridding forward model, [B][Lmax][n] (lines beyond L_b zero)."""
    import numpy as np
    import torch

    from synth.phantom import ground_truth_volume

    S = case.n_spec
    shp = B.nu_shape(plan)
    y = np.zeros(shp, dtype=np.complex64)
    for b in range(case.n_blades):
        t = 0.0 if case.n_time == 1 else float(case.blade_time[b])
        pb = B.Plan(case.n, S, 1, case.angle_rad[b:b + 1], case.lines[b:b + 1], None, case.spec_shift_px)
        w, f = case.layers_at(t)
        gt = torch.from_numpy(ground_truth_volume(w, f, S)[None].astype(np.complex64)).cuda()
        L = int(case.lines[b])
        y[b, :L] = B.vp_nu_forward(pb, gt).cpu().numpy()[0, :L] + case.sigma * case.noise[b][:L, :]
    return y


def nu_leg(B, name, steps, warmup):
    """The fit on blade-aligned samples (gridding in place of the masked Cartesian DFT) on a
    workload's geometry: step throughput, per-stage times, the HBM roofline of the dominant
    stage and the PSNR of the fit against the phantom."""
    import numpy as np
    import torch

    from synth import configs

    case = configs.CONFIGS[name]()
    plan = B.Plan.from_geometry(case.geometry())
    y = gpu_samples(case, plan, B)
    opts = B.vp_options_default(**configs.config_options(case), device=0)
    sess = B.NuSession(plan, y, opts)
    sess.step(warmup, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sess.step(steps, use_graph=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    stages = sess.stage_times(max(3, steps // 4))
    sess.close()
    # algorithmic HBM bytes per launch of each blade-aligned kernel (complex64 = 8 bytes),
    # per blade: the forward row pass reads the blade image(s) and writes the n image rows
    # of the 2n x 2n grid; the forward column pass reads those rows and writes the grid;
    # interp reads the grid points within W/2 of the blade's lattice (a (2n + 6) x
    # (2L + 6) strip) and per sample y and the phase, and writes the residual and the
    # spread's input; spread reads that input and writes the grid; the inverse column pass
    # reads the grid and writes the image rows; the inverse row pass reads them and writes
    # the blade image
    n, Bn = case.n, case.n_blades
    M = 2 * n
    L = int(np.max(case.lines))
    ns = Bn * L * n
    parts = 2 if case.n_time > 1 else 1
    strip = min(M * M, (M + 6) * (2 * L + 6))
    per = {"rows_fwd": 8 * Bn * (parts * n * n + n * M), "cols_fwd": 8 * Bn * (n * M + M * M),
           "interp": 8 * Bn * strip + 32 * ns, "spread": 8 * Bn * M * M + 8 * ns,
           "cols_inv": 8 * Bn * (M * M + n * M), "rows_inv": 8 * Bn * (n * M + n * n)}
    dom = max(per, key=lambda k: stages[k])
    ach = per[dom] / (stages[dom] * 1e-3) / 1e9
    # quality: a whole fit from zero at the workload's step count
    r = B.vp_nu_reconstruct(plan, y, opts)
    if case.n_time == 1:
        truth = np.asarray(sum(case.layers_at(0.0)), dtype=np.complex64)[None]
    else:
        truth = np.stack([sum(case.layers_at(k / (case.n_time - 1))) for k in range(case.n_time)])
    p_fit = B.vp_psnr(torch.from_numpy(r["proj"]).cuda(),
                      torch.from_numpy(truth.astype(np.complex64)).cuda())[0].cpu().numpy()
    return {"workload": f"{name} geometry, blade-aligned samples (Kaiser-Bessel gridding, width 6, grid 2n)",
            "value": round(case.n_blades * steps / el, 1), "unit": "blade fwd+adjoint/s",
            "ms_per_step": round(el * 1e3 / steps, 5), "steps": steps,
            "stage_ms": {k: round(v, 5) for k, v in stages.items()},
            "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
                         "kernel_ms": round(stages[dom], 5), "algorithmic_bytes_per_launch": per[dom]},
            "quality": {"psnr_db": round(float(np.mean(p_fit)), 2), "steps": case.n_steps}}


def shard_leg(B, name, gpus, steps, warmup):
    """One GPU's share of a spectral split of one volume over `gpus` GPUs (the sharding
    design): the workload's geometry restricted to the last S / gpus bins (the largest
    shifts, so the widest halos), stepped as one slice. Each GPU would also run the blade
    DFT passes on the all-reduced blade images (counted here, redundantly per GPU) and
    swap one TV halo plane with each spectral neighbour; the all-reduce itself is not
    run (one GPU) and is reported as an estimate over xGMI."""
    import numpy as np
    import torch

    from synth import configs

    case = configs.CONFIGS[name]()
    g = case.geometry()
    S = case.n_spec
    share = S // gpus
    g["n_spec"] = share
    g["spec_shift_px"] = np.asarray(g["spec_shift_px"])[S - share:]
    plan = B.Plan.from_geometry(g)
    rng = np.random.default_rng(case.seed)
    y = ((rng.standard_normal(plan.blade_shape) + 1j * rng.standard_normal(plan.blade_shape))
         * plan.masks()).astype(np.complex64)
    opts = B.vp_options_default(n_steps=case.n_steps, tv_weight=case.tv_weight, lr=case.lr, device=0, autotune=1)
    plan.tune(opts)
    sess = B.Session(plan, y, opts)
    sess.step(warmup, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sess.step(steps, use_graph=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    stages = sess.stage_times(max(3, steps // 4))
    sess.close()
    # ring all-reduce of the B blade images (complex64) over 7 xGMI links of about 153 GB/s
    ar_bytes = 8 * case.n_blades * case.n * case.n
    ring_us = 2 * (gpus - 1) / gpus * ar_bytes / 153e9 * 1e6
    return {"workload": f"{name} geometry, bins {S - share}..{S - 1} of {S} (one GPU of a {gpus}-way spectral split)",
            "ms_per_step": round(el * 1e3 / steps, 5), "steps": steps,
            "stage_ms": {k: round(v, 5) for k, v in stages.items()},
            "allreduce_bytes": ar_bytes, "allreduce_ring_us_estimate": round(ring_us, 1),
            "note": "measured on one GPU; the collective is an estimate, not run"}


def _digest(r):
    """A result's rendered images (hashed) and objective: equal digests are bitwise equal
    results as a client receives them (the renders are fixed sums of the volume's bins)."""
    h = hashlib.sha256()
    for k in ("proj", "water", "fat"):
        h.update(r[k].tobytes())
    return h.hexdigest(), r["final_loss"]


def served_leg(B, n_req, steps_static, steps_dynamic, seed=5000, slots=8):
    """A Poisson request stream of mixed static/dynamic reconstructions through the server."""
    import numpy as np
    import torch

    from synth import configs

    cases = [configs.serving_request(i, seed) for i in range(n_req)]
    probs = []
    for k, c in enumerate(cases):
        probs.append(_slice_problem(c, B))
        if (k + 1) % 50 == 0:
            progress(f"served: {k + 1} of {n_req} requests simulated")
    opts = [B.vp_options_default(n_steps=steps_static if c.n_time == 1 else steps_dynamic,
                                 tv_weight=c.tv_weight, lr=c.lr) for c in cases]
    B.vp_reconstruct(probs[0][0], probs[0][1], B.vp_options_default(n_steps=2))
    _warm_plans(probs, B)
    # every pass returns what a client of the served stream receives: the rendered image,
    # water and fat images and the objective (the volume stays on the device)
    t0 = time.perf_counter()
    solo = [_digest(B.vp_reconstruct(p, y, o, volume=False)) for (p, y), o in zip(probs, opts)]
    t_plain = time.perf_counter() - t0
    progress(f"served: plain loop {t_plain:.1f} s")
    # the plain loop as the baseline definition has it: one request at a time, kernels
    # launched eagerly (no graph), nothing overlapped
    t0 = time.perf_counter()
    eager = []
    for (p, y), o in zip(probs, opts):
        sess = B.Session(p, y, o)
        sess.step(o.n_steps, use_graph=False)
        obj = sess.objective()[0]
        r = sess.read(volume=False)
        sess.close()
        r["final_loss"] = obj
        eager.append(_digest(r))
    t_eager = time.perf_counter() - t0
    progress(f"served: eager plain loop {t_eager:.1f} s")
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    # closed loop: everything submitted at once gives the server's capacity
    srv = B.Server(device=0, hbm_budget=budget, max_slots=slots)
    t0 = time.perf_counter()
    ids = [srv.submit(p, y, o) for (p, y), o in zip(probs, opts)]
    closed = [_digest(srv.wait(i, volume=False)) for i in ids]
    t_closed = time.perf_counter() - t0
    srv.close()
    progress(f"served: closed loop {t_closed:.1f} s")
    capacity = n_req / t_closed
    rate = 0.7 * capacity
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_req)
    srv = B.Server(device=0, hbm_budget=budget, max_slots=slots)
    t0 = time.perf_counter()
    ids = []
    for k, ((p, y), o) in enumerate(zip(probs, opts)):
        target = t0 + float(np.sum(gaps[:k + 1]))
        now = time.perf_counter()
        if target > now:
            time.sleep(target - now)
        ids.append(srv.submit(p, y, o))
    served = [_digest(srv.wait(i, volume=False)) for i in ids]
    t_open = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    same = solo == served and solo == closed and [d[0] for d in solo] == [d[0] for d in eager]
    full = steps_static == 200 and steps_dynamic == 800
    return {"workload": f"{n_req} requests (seeds {seed}+i): n 128-384, S 16-64, 8-32 blades, T in {{1,8,16}}; "
                        f"{steps_static} steps static / {steps_dynamic} dynamic"
                        + ("" if full else " (the served mix's own 200 / 800 steps scaled down so that the three "
                                           "passes over the stream fit the benchmark's few minutes; "
                                           "bench.py --serve-steps 200 800 runs them in full)"),
            "plain_loop_s": round(t_plain, 3), "plain_loop_rps": round(n_req / t_plain, 3),
            "plain_loop_eager_s": round(t_eager, 3),
            "speedup_vs_plain_loop": round(t_plain / t_closed, 3),
            "speedup_vs_plain_loop_eager": round(t_eager / t_closed, 3),
            "plain_loops": "plain_loop: vp_reconstruct per request (upload, graph-replayed steps, objective, "
                           "read-back of the rendered image, water and fat images); plain_loop_eager: the same "
                           "with kernels launched eagerly, no graph; every pass reads back the same renders "
                           "and objective, and their digests must agree bit for bit",
            "closed_loop_rps": round(capacity, 3), "arrival_rate_rps": round(rate, 3),
            "open_loop_s": round(t_open, 3), "p50_ms": round(st["p50_us"] / 1e3, 2),
            "p99_ms": round(st["p99_us"] / 1e3, 2), "served_rps": round(st["throughput_rps"], 3),
            "served_equals_solo_bitwise": bool(same), "max_slots": slots}


def copy_probe():
    """A plain device copy of known size, for scaling HBM byte counters."""
    import torch

    n = 1 << 28  # 1 GiB of float32 per buffer
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "launches": 5}))


# Source files of each kernel family (plus the shared device headers).
KERNEL_SOURCES = {"k_gather": ["k_gather.hip", "update.h"], "k_gather_res": ["k_gather_res.hip", "update.h"],
                  "k_update": ["k_gather.hip", "update.h"],
                  "k_project": ["k_project.hip"],
                  "k_rows": ["k_fft.hip"], "k_cols": ["k_fft.hip"]}


def kernel_digest(kernel=None):
    """sha256 (first 16 hex) over the sources of one kernel family (by kernel name, e.g.
    "k_gather<1>") and the shared device headers, or over every device source."""
    csrc = os.path.join(ROOT, "paper_2311_13177_amd", "csrc")
    fam = None if kernel is None else kernel.split("<")[0]
    if fam in KERNEL_SOURCES:
        names = sorted(KERNEL_SOURCES[fam]) + ["kcommon.h"]
    else:
        names = sorted(f for f in os.listdir(csrc) if f.startswith("k") and f.endswith((".hip", ".h")))
    names.append("vp_internal.h")
    h = hashlib.sha256()
    for f in names:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


TILE_FIELDS = ("proj_rows", "proj_parts", "gath_rows", "gath_bins", "upd_bins", "gath_waves", "proj_waves",
               "gath_resident")
# The tile fields that select a kernel family's variant (the DFT passes have none).
FAMILY_TILES = {"k_gather": ("gath_rows", "gath_bins", "upd_bins", "gath_waves", "gath_resident"),
                "k_gather_res": ("gath_rows", "gath_bins", "upd_bins", "gath_waves", "gath_resident"),
                "k_project": ("proj_rows", "proj_parts", "proj_waves")}


def counters_for(workload, kernel_name, tiles=None):
    """HBM bytes per launch (scaled FETCH_SIZE + WRITE_SIZE) from the committed counter
    summary of this workload, or None once the kernel's sources have changed since, or
    when the counters were taken on another variant (tile shape) than the one timed."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    entry = data.get(f"{workload}/{kernel_name}")
    if not entry or entry.get("kernels_sha") != kernel_digest(kernel_name):
        return None
    fam = kernel_name.split("<")[0]
    if tiles is not None and fam in FAMILY_TILES:
        now = dict(zip(TILE_FIELDS, tiles))
        then = entry.get("tiles") or {}
        if any(then.get(f) != now.get(f) for f in FAMILY_TILES[fam]):
            return None
    return entry.get("bytes_per_launch")


def quality(case, plan, B, y, rec):
    """PSNR on magnitudes (HIP reduction) of the reconstruction and of the Section 6
    baseline against the phantom: static, the projection against W + F and the baseline
    over all blades; dynamic, the knot frames against the phantom at the knot times and
    the five-blade baseline frames against it at the blade times (means over frames)."""
    import numpy as np
    import torch

    def truth(tau):
        w, f = case.layers_at(float(tau))
        return (w + f).astype(np.complex64)

    d_y = torch.from_numpy(y).cuda()
    if case.n_time == 1:
        t = torch.from_numpy(truth(0.0)[None]).cuda()
        base = B.vp_baseline(plan, d_y)
        kind, times = "coverage-weighted average of all blades", None
    else:
        t = torch.from_numpy(np.stack([truth(k / (case.n_time - 1)) for k in range(case.n_time)])).cuda()
        base = B.vp_baseline(plan, d_y, window=5, first_frame=0, n_frames=case.n_blades)
        times = case.blade_time
        kind = "coverage-weighted average of the 5 most recent blades per frame"
    ours = torch.from_numpy(np.ascontiguousarray(rec["proj"]).astype(np.complex64)).cuda()
    p_ours = B.vp_psnr(ours, t)[0].cpu().numpy()
    tb = t if times is None else torch.from_numpy(np.stack([truth(tau) for tau in times])).cuda()
    p_base = B.vp_psnr(base, tb)[0].cpu().numpy()
    return {"psnr_db": round(float(np.mean(p_ours)), 2), "baseline_psnr_db": round(float(np.mean(p_base)), 2),
            "baseline": kind, "frames": int(p_ours.shape[0]), "baseline_frames": int(p_base.shape[0]),
            "steps": case.n_steps}


def measure_workload(case, B, steps, warmup, tiles=None):
    """Autotuned steps of one workload (or steps of the tile shape given): throughput,
    per-stage times and the roofline of the dominant stage's kernel."""
    import torch

    plan = B.Plan.from_geometry(case.geometry())
    y = gpu_measurements(case, plan, B)
    t0 = time.perf_counter()
    if tiles is None:
        opts = B.vp_options_default(n_steps=case.n_steps, tv_weight=case.tv_weight, lr=case.lr, device=0,
                                    autotune=1)
        # tile shapes picked by the autotuner (recorded for this plan's sizes; not timed below)
        tiles = plan.tune(opts)
    else:
        opts = B.vp_options_default(n_steps=case.n_steps, tv_weight=case.tv_weight, lr=case.lr, device=0,
                                    tiles=tiles)
        tiles = plan.tiles(opts)
    tune_s = time.perf_counter() - t0

    # whole reconstruction wall time (upload, n_steps graph-replayed steps, objective, download)
    t0 = time.perf_counter()
    rec = B.vp_reconstruct(plan, y, opts)
    recon_s = time.perf_counter() - t0
    assert math.isfinite(rec["final_loss"])

    sess = B.Session(plan, y, opts)
    sess.step(warmup, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sess.step(steps, use_graph=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_per_step = el * 1e3 / steps
    value = case.n_blades * steps / el

    stages = sess.stage_times(steps)
    sess.close()
    qual = quality(case, plan, B, y, rec)
    stage_bytes, stage_flops, parts = algorithmic(case)
    dom = max(stages, key=lambda k: stages[k])
    dur_s = stages[dom] * 1e-3
    kernel_names = {"project": "k_project", "rows_fwd": "k_rows<-1>", "cols": "k_cols", "rows_inv": "k_rows<1>",
                    "gather_update": ("k_gather_res" if tiles[7] else "k_gather<1>") if tiles[4] == 0
                    else "k_gather<0>+k_update"}
    bytes_l = stage_bytes[dom]
    flops_l = stage_flops.get(dom, 0)
    ai = flops_l / bytes_l
    if ai > FP32_VALU_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9):
        ach = flops_l / dur_s / 1e12
        roof = {"bound": "alu", "achieved": round(ach, 3), "peak": FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / FP32_VALU_TFLOPS, 4)}
    else:
        ach = bytes_l / dur_s / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4)}
    roof["traffic"] = counters_for(case.name, kernel_names[dom], tiles)
    roof["kernel"] = kernel_names[dom]
    roof["kernel_ms"] = round(stages[dom], 5)
    roof["algorithmic_bytes_per_launch"] = bytes_l
    return {
        "value": round(value, 1),
        "ms_per_step": round(ms_per_step, 5),
        "steps": steps,
        "config": {"workload": case.name, "n": case.n, "n_spec": case.n_spec, "n_time": case.n_time,
                   "n_blades": case.n_blades, "lines": int(case.lines[0]), "steps_per_recon": case.n_steps,
                   "optimizer": "adam", "schedule": "all blades per step",
                   "tiles": dict(zip(TILE_FIELDS, tiles)),
                   "tune_s": round(tune_s, 4)},
        "recon_wall_s": round(recon_s, 4),
        "stage_ms": {k: round(v, 5) for k, v in stages.items()},
        "step_hbm_bytes_algorithmic": int(sum(stage_bytes.values())),
        "roofline": roof,
        "quality": qual,
    }


def main(argv=None):
    args = parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design, not a measured path", file=sys.stderr)
        return 2
    if args.copy_probe:
        copy_probe()
        return 0
    import numpy as np
    import torch

    from paper_2311_13177_amd import binding as B
    from synth import configs

    torch.cuda.set_device(0)
    case = configs.CONFIGS[args.config]()
    progress(f"headline {case.name}")
    forced = None if args.tiles is None else tuple(int(x) for x in args.tiles.split(","))
    m = measure_workload(case, B, args.steps, args.warmup, forced)

    out = {
        "metric": METRIC,
        "value": m["value"],
        "unit": "blade fwd+adjoint/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": m["config"],
        "recon_wall_s": m["recon_wall_s"],
        "stage_ms": m["stage_ms"],
        "step_hbm_bytes_algorithmic": m["step_hbm_bytes_algorithmic"],
        "roofline": m["roofline"],
        "quality": m["quality"],
    }
    if not args.no_static and case.name != "static_256":
        # the 256^2 static workload: its 48 MiB state fits the Infinity Cache, so HBM does
        # not bind it (the headline is the dynamic workload, whose state does not fit)
        progress("static_256")
        d = measure_workload(configs.CONFIGS["static_256"](), B, max(50, args.steps), args.warmup)
        out["static_256"] = d
    if not args.no_kplanes:
        progress("kplanes_192")
        out["kplanes_192"] = kplanes_leg(B, max(20, args.steps // 8), 3)
    if not args.no_nu:
        progress("nu_256")
        out["nu_256"] = nu_leg(B, "static_256", max(20, args.steps // 4), 3)
    if not args.no_shard:
        progress("shard_share_192")
        out["shard_share_192"] = shard_leg(B, "dynamic_192", 8, max(20, args.steps // 4), 3)
    if not args.no_batch:
        progress("batched")
        out["batched"] = batched_leg(B, args.batch_slices, args.batch_steps)
    if not args.no_serve:
        progress("served")
        out["served"] = served_leg(B, args.serve_requests, args.serve_steps[0], args.serve_steps[1])
    if not args.no_cpu:
        progress("cpu_baseline")
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_seconds)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
