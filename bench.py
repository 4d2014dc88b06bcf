#!/usr/bin/env python3
"""Benchmark of the generalized MBO iteration (Osting & Wang, arXiv:1711.01365).

Workload (one "step"): Algorithm 1 on an n = 3 field over a 512 x 512 periodic
grid of [0,1)^2, initial values Haar-random in O(3) per point (seed 1),
tau = 2e-4, 200 iterations, FP32 diffusion and projection with FP64 re-projection
of points whose smallest singular value is below 1e-3.  Each step restores the
initial field (a device copy) and runs the 200 iterations as one captured HIP
graph, with the Lyapunov energy, det-flip and fallback logs copied back once.
The plan's launch shapes are chosen by its autotuner (mbo_plan_autotune) before
the timed region; the JSON line records them.  The same workload in full FP64
is timed beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  `value` is point-iterations per second (points x
iterations x steps / seconds) on one GPU.  `roofline` prices the dominant kernel
(the row pass) by its algorithmic bytes per launch -- one read and one write of
the n x n FP32 field, 72 bytes per point -- over its average duration, taken
from HIP start/stop events recorded by each dispatch in three more steps run
right after the timed ones (launched directly, since events inside a captured
graph cannot be timed).  `cpu_baseline` is
the FP64 CPU oracle on a bounded sample (the first iterations of the same
workload).  Beside the main line: a 2048^2 bandwidth control (the same
kernels on a field 16x larger), the 3-D configuration (n = 3, 128^3, 100
iterations, FP32 + fallback), the batched configuration (64 fields of mixed n,
grid and tau, 50 iterations in one graph; FP32 autotuned, FP32 with the fixed
launch rules, FP64), the volume-preserving method of Section 7 (n = 3, 512^2
Haar, 200 iterations; and the paper's example, the star-shaped defect with
n = 2 on 1024^2, tau = 8 dx, 100 iterations; FP32 + fallback, the SO(n) volume
of the initial field held fixed) and the gradient of 50 unrolled steps (n = 3,
256^2, FP32 + fallback and FP64), forward and backward time; the paper's three
flat-torus examples (n = 2, 1024^2, FP32 + fallback) with their end states;
the relaxed gradient flows GD-1 / GD-3 (n = 3, 512^2, 200 steps); the sphere of
Section 6.2 (closest-point band, dx = 0.05, p = 3, tau = 0.005, 3.3 M samples,
20 MBO steps, FP32 + fallback and FP64, in sample-steps per second); and the
volume-preserving sphere of Section 7 (tau = 0.01, 5.1 M samples, 20 steps).
With --peanut, the peanut of Section 6.3 (116.5 M samples, 10 steps) is added.

    python bench.py --volume-only [--steps K] [--warmup W]

runs only the two volume-preserving legs (for profiling them), and

    python bench.py --surface-only [--peanut] [--steps K]

only the surface legs.

    python bench.py --copy-calibration

runs only a plain device copy of 256 MiB (ten times), the reference the
hardware byte counters are scaled by.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "row_fast_n3_512x512_f32fb_traffic.txt")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# sources that decide the row pass's code and launch shape (its traffic)
ROW_PASS_SOURCES = ("mbo_device.hpp", "mbo_kernels.hpp", "mbo_internal.hpp", "mbo_fast.hpp",
                    "mbo_fast_launch.hpp", "mbo_fast_f32.hip", "mbo_api.cpp")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1711_01365_amd", "csrc")
    for f in ROW_PASS_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def read_traffic():
    """HBM traffic of the row pass per launch from the committed counter summary,
    or None when it is missing or was taken on different kernel sources."""
    if not os.path.exists(PROFILE_TRAFFIC):
        return None
    kv = {}
    for line in open(PROFILE_TRAFFIC):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(kv["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration():
    import torch
    n = 64 * 1024 * 1024  # floats: 256 MiB
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 10}))


def launch_shape(w, precision, path, tuning, autotune):
    """Launch shape of the iteration's kernels.  The band-limited row pass has a
    fixed shape per (n, row length) (512 points per workgroup, or one long row);
    the heat tile width and the XCD order are tuned.  The general path reports
    its tuned row-pass shape."""
    from paper_1711_01365_amd import mbo
    if path[0] == mbo.PATH_GENERIC:
        return {"rows_per_row_workgroup": tuning[0], "row_workgroup_threads": tuning[1],
                "lines_per_heat_workgroup": tuning[2], "xcd_tile_order": tuning[3], "autotuned": bool(autotune)}
    L, n = w.grid[-1], w.n
    tn, pl = L // 8, (n * n + 1) // 2
    rows = 1 if L >= 512 else 512 // L
    if L <= 512:
        threads = 512
    else:
        ntmax = 768 if (precision != mbo.F64 and n == 3) else 1024
        threads = max(512, min(rows * pl * tn, ntmax // tn * tn))
    return {"rows_per_row_workgroup": rows, "row_workgroup_threads": threads,
            "columns_per_heat_workgroup": tuning[2], "xcd_tile_order": tuning[3], "autotuned": bool(autotune)}


def run_gpu(w, precision, steps, warmup, timing_steps, autotune=True):
    """Timed region: `steps` steps through the captured graph (the product path).
    Then `timing_steps` more steps with per-kernel HIP events (direct launches)."""
    import numpy as np
    import torch
    from paper_1711_01365_amd import mbo

    dt = torch.float64 if precision == mbo.F64 else torch.float32
    A0 = torch.tensor(w.field(), dtype=dt, device="cuda")
    A = A0.clone()
    plan = mbo.Plan(w.grid, w.n, w.tau, precision=precision)
    tuning = plan.autotune() if autotune else plan.tuning()
    path = plan.path()
    for _ in range(warmup):
        A.copy_(A0)
        plan.iterate(A, w.iters)
    torch.cuda.synchronize()
    logs = None
    t0 = time.perf_counter()
    for _ in range(steps):
        A.copy_(A0)
        logs = plan.iterate(A, w.iters)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    row_us, col_us = [], []
    if timing_steps:
        plan.set_timing(True)
        for k in range(timing_steps + 1):
            A.copy_(A0)
            plan.iterate(A, w.iters)
            if k:  # the first one warms the direct-launch path
                r, c, _k = plan.last_timing()
                row_us.append(r)
                col_us.append(c)
        torch.cuda.synchronize()
    plan.close()
    return {
        "seconds": sec,
        "value": w.points * w.iters * steps / sec,
        "ms_per_step": 1000.0 * sec / steps,
        "row_us": float(np.mean(row_us)) if row_us else None,
        "heat_us": float(np.mean(col_us)) if col_us else None,
        "energy_first_last": [float(logs["energy"][0][0]), float(logs["energy"][0][-1])],
        "fallbacks_total": int(logs["fallbacks"][0].sum()),
        "launch_shape": launch_shape(w, precision, path, tuning, autotune),
        "flips_first": int(logs["flips"][0][0]),
        "path": {"kind": {0: "generic", 1: "full", 2: "banded"}[path[0]], "half_width": path[1],
                 "stored_modes": path[2]},
    }


def run_control_2048():
    """n = 3 on 2048^2 (20 iterations, FP32 + fallback): the same kernels on a
    field 16x larger, where the passes stream from HBM; kernel times from
    dispatch events and their algorithmic bandwidth."""
    from paper_1711_01365_amd import inputs, mbo
    w = inputs.CONTROL_2048
    r = run_gpu(w, mbo.F32_F64FALLBACK, 3, 1, timing_steps=2)
    bpl = 2 * w.n * w.n * 4 * w.points
    return {"workload": "n3_2048x2048_haar_20it_f32_f64fallback", "value": r["value"],
            "unit": "point-iterations/s", "row_us": r["row_us"], "heat_us": r["heat_us"],
            "bytes_per_launch": bpl,
            "row_GBps": bpl / (r["row_us"] * 1e-6) / 1e9, "heat_GBps": bpl / (r["heat_us"] * 1e-6) / 1e9}


def run_3d(steps, warmup):
    """The 3-D configuration (n = 3, 128^3, 100 iterations, FP32 + FP64 fallback)
    through the captured graph; point-iterations per second.  Beside it the two
    passes of an iteration (the row pass along the last axis with the
    projection, the plane pass over the other two axes), timed with dispatch
    events, and their algorithmic bandwidth (the field read once and written
    once per pass)."""
    from paper_1711_01365_amd import inputs, mbo
    w = inputs.NORMAL_128_3D
    r = run_gpu(w, mbo.F32_F64FALLBACK, steps, warmup, timing_steps=2)
    bpl = 2 * w.n * w.n * 4 * w.points
    # what the passes move: the kept x modes of the packed planes of every
    # (z, y) row, read and written by both passes, and the row pass's det signs
    pl = (w.n * w.n + 1) // 2
    spectra = pl * r["path"]["stored_modes"] * (w.points // w.grid[2]) * 8
    moved_row, moved_plane = 2 * spectra + 2 * w.points, 2 * spectra
    return {"workload": "n3_128x128x128_normal_tau5e-4_100it_f32_f64fallback",
            "value": r["value"], "unit": "point-iterations/s", "ms_per_run": r["ms_per_step"],
            "row_us": r["row_us"], "plane_us": r["heat_us"], "bytes_per_launch": bpl,
            "row_GBps": bpl / (r["row_us"] * 1e-6) / 1e9, "plane_GBps": bpl / (r["heat_us"] * 1e-6) / 1e9,
            "moved_bytes_per_launch_model": {"row_pass": moved_row, "plane_pass": moved_plane},
            "moved_GBps": {"row_pass": moved_row / (r["row_us"] * 1e-6) / 1e9,
                           "plane_pass": moved_plane / (r["heat_us"] * 1e-6) / 1e9},
            "path": r["path"], "fallbacks_total": r["fallbacks_total"]}


def run_volume(w, steps, warmup):
    """Volume-preserving MBO (Section 7) on workload w, FP32 + FP64 fallback,
    through its captured graph, n_plus = the SO(n) points of A_0; beside it the
    plain iteration of the same workload on the same plan."""
    import numpy as np
    import torch
    from paper_1711_01365_amd import mbo
    A0 = torch.tensor(w.field(), dtype=torch.float32, device="cuda")
    A = A0.clone()
    plan = mbo.Plan(w.grid, w.n, w.tau, precision=mbo.F32_F64FALLBACK)
    plan.autotune()

    def timed(fn):
        for _ in range(warmup):
            A.copy_(A0)
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            A.copy_(A0)
            fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    logs = {}

    def vol():
        logs.update(plan.iterate_volume(A, w.iters))

    sec = timed(vol)
    n_plus = int(logs["n_plus"][0])
    E = logs["energy"][0]
    sec_plain = timed(lambda: plan.iterate(A, w.iters, logs=False))
    plan.close()
    return {"workload": w.name + "_tau%g_%dit_f32_f64fallback" % (w.tau, w.iters),
            "value": w.points * w.iters * steps / sec, "unit": "point-iterations/s",
            "us_per_iteration": 1e6 * sec / (steps * w.iters),
            "plain_mbo_us_per_iteration": 1e6 * sec_plain / (steps * w.iters),
            "n_plus": n_plus, "energy_first_last": [float(E[0]), float(E[-1])],
            "energy_nonincreasing": bool(np.all(np.diff(E[1:]) <= 1e-5 * np.abs(E[1:-1])))}


def run_examples(steps):
    """The paper's three flat-torus examples (n = 2, 1024^2, FP32 + FP64
    fallback, their iteration counts) through the captured graph: rate and the
    end state (points in SO(2), SO(2) index along x and y loops)."""
    import numpy as np
    import torch
    from paper_1711_01365_amd import inputs, mbo
    out = {}
    for w in (inputs.EXAMPLE_STAR, inputs.EXAMPLE_LINES, inputs.EXAMPLE_WINDING):
        A0 = torch.tensor(w.field(), dtype=torch.float32, device="cuda")
        A = A0.clone()
        plan = mbo.Plan(w.grid, w.n, w.tau, precision=mbo.F32_F64FALLBACK)
        plan.autotune()
        A.copy_(A0)
        plan.iterate(A, w.iters)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            A.copy_(A0)
            lg = plan.iterate(A, w.iters)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        wx, wy = plan.so2_index(A)
        a = A.double().cpu().numpy()
        det = a[0, 0] * a[1, 1] - a[0, 1] * a[1, 0]
        plan.close()
        out[w.name] = {"tau": w.tau, "iterations": w.iters,
                       "value": w.points * w.iters * steps / sec, "unit": "point-iterations/s",
                       "us_per_iteration": 1e6 * sec / (steps * w.iters),
                       "so2_points_end": int((det > 0).sum()),
                       "index_end": [sorted(set(np.rint(wx[0]).astype(int).tolist())),
                                     sorted(set(np.rint(wy[0]).astype(int).tolist()))],
                       "energy_first_last": [float(lg["energy"][0][0]), float(lg["energy"][0][-1])]}
    return out


def run_relaxed(steps):
    """The relaxed gradient flows GD-1 and GD-3 (n = 3, 512^2 Haar field,
    FP32 + FP64 fallback, eps = 4 dx, dt = 0.1 eps^2, 200 steps) through their
    captured graph: step rate and the energy before / after."""
    import torch
    from paper_1711_01365_amd import inputs, mbo
    w = inputs.HAAR_512
    eps = 4.0 / w.grid[0]
    dt = 0.1 * eps * eps
    K = 200
    A0 = torch.tensor(w.field(), dtype=torch.float32, device="cuda")
    A = A0.clone()
    plan = mbo.Plan(w.grid, w.n, w.tau, precision=mbo.F32_F64FALLBACK)
    plan.autotune()
    out = {}
    for name, kind in (("gd1", mbo.GD1), ("gd3", mbo.GD3)):
        A.copy_(A0)
        plan.relaxed_flow(A, K, kind, eps, dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            A.copy_(A0)
            plan.relaxed_flow(A, K, kind, eps, dt)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        out[name] = {"workload": "n3_512x512_haar_eps%.4g_dt%.3g_%dsteps_f32_f64fallback" % (eps, dt, K),
                     "value": w.points * K * steps / sec, "unit": "point-steps/s",
                     "us_per_step": 1e6 * sec / (steps * K),
                     "energy_first_last": [plan.relaxed_energy(A0, kind, eps), plan.relaxed_energy(A, kind, eps)]}
    plan.close()
    return out


def run_surface(steps, precisions=None):
    """The sphere experiment of Section 6.2 (unit sphere, dx = 0.05, p = 3,
    tau = 0.005, eps = 1e-6, n = 3, 20 MBO steps from the printed matrices by
    octant): sample-steps/s of the closest-point MBO iteration, the time of one
    diffusion step, and the SO^-(3) sample count before / after."""
    import numpy as np
    import torch
    from paper_1711_01365_amd import inputs, mbo
    w = inputs.SPHERE_PAPER
    out = {}
    for name, prec in (precisions or (("f32_f64fallback", mbo.F32_F64FALLBACK), ("f64", mbo.F64))):
        t0 = time.perf_counter()
        s = mbo.SphereSurface(w.R, w.dx, w.p, w.tau, w.eps, w.n, precision=prec)
        setup = time.perf_counter() - t0
        xq, xc, wts = s.points()
        dt = torch.float64 if prec == mbo.F64 else torch.float32
        A0 = torch.tensor(inputs.sphere_octant_field(xc), dtype=dt, device="cuda")
        A = A0.clone()
        B = torch.empty_like(A)
        s.iterate(A, 1)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            A.copy_(A0)
            s.iterate(A, w.iters)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(5):
            s.diffuse(A0, B)
        ev1.record()
        torch.cuda.synchronize()
        det = np.linalg.det(np.moveaxis(A.double().cpu().numpy(), 2, 0))
        x, y, z = xc
        out[name] = {"workload": "%s_n3_%dit_%s" % (w.name, w.iters, name),
                     "value": s.m * w.iters * steps / sec, "unit": "sample-steps/s",
                     "samples": s.m, "band_cells": s.cells, "grid": s.grid,
                     "us_per_step": 1e6 * sec / (steps * w.iters),
                     "diffuse_us": 1e3 * ev0.elapsed_time(ev1) / 5, "setup_s": setup,
                     "so3minus_samples_first_last": [int(((x < 0) & (y < 0) & (z > 0)).sum()), int((det < 0).sum())]}
        s.close()
    return out


def run_surface_volume(steps):
    """Volume-preserving MBO on the sphere of Section 7 (dx = 0.05, p = 3,
    tau = 0.01, eps = 1e-6, n = 3, FP32 + fallback, 20 steps from the printed
    matrices by octant, V = the initial SO(3) volume): sample-steps/s and the
    volume kept."""
    import numpy as np
    import torch
    from paper_1711_01365_amd import inputs, mbo
    w = inputs.SPHERE_VOLUME_PAPER
    s = mbo.SphereSurface(w.R, w.dx, w.p, w.tau, w.eps, w.n, precision=mbo.F32_F64FALLBACK)
    xq, xc, wts = s.points()
    W = s.volume_weights()
    A0 = torch.tensor(inputs.sphere_octant_field(xc), dtype=torch.float32, device="cuda")
    A = A0.clone()
    V, _ = s.iterate_volume(A, 1)  # warm-up; V = weight of the samples with det >= 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        A.copy_(A0)
        s.iterate_volume(A, w.iters, V)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    det = np.linalg.det(np.moveaxis(A.double().cpu().numpy(), 2, 0))
    kept = int(W[det > 0].sum())
    out = {"workload": "%s_n3_%dit_f32_f64fallback" % (w.name, w.iters),
           "value": s.m * w.iters * steps / sec, "unit": "sample-steps/s", "samples": s.m, "grid": s.grid,
           "us_per_step": 1e6 * sec / (steps * w.iters), "volume_target": V, "volume_end": kept,
           "volume_within_one_sample": bool(V <= kept < V + int(W.max()))}
    s.close()
    return out


def run_peanut(steps):
    """The peanut experiment of Section 6.3 (dx = 0.04, p = 4, tau = 0.032,
    eps = 1e-6, n = 3, FP32 + fallback, 10 MBO steps from the printed matrices):
    sample-steps/s, the host time of the sample set, and the flips per step."""
    import torch
    from paper_1711_01365_amd import inputs, mbo
    w = inputs.PEANUT_PAPER
    t0 = time.perf_counter()
    s = mbo.PeanutSurface(w.dx, w.p, w.tau, w.eps, w.n, precision=mbo.F32_F64FALLBACK)
    setup = time.perf_counter() - t0
    xq, xc, wts = s.points()
    del xq, wts
    A0 = torch.tensor(inputs.peanut_field(xc), dtype=torch.float32, device="cuda")
    A = A0.clone()
    s.iterate(A, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        A.copy_(A0)
        s.iterate(A, w.iters)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    A.copy_(A0)
    fl = s.iterate(A, 3, flips=True)
    out = {"workload": "%s_n3_%dit_f32_f64fallback" % (w.name, w.iters),
           "value": s.m * w.iters * steps / sec, "unit": "sample-steps/s", "samples": s.m, "band_cells": s.cells,
           "grid": s.grid, "us_per_step": 1e6 * sec / (steps * w.iters), "setup_s": setup,
           "flips_first_steps": [int(f) for f in fl]}
    s.close()
    return out


def run_adjoint(precision, reps):
    """Gradients of K = 50 unrolled steps (n = 3, 256^2, checkpoint every 10):
    forward and backward wall time of the autograd function."""
    import torch
    from paper_1711_01365_amd import inputs, mbo
    from paper_1711_01365_amd.autograd import unrolled_mbo
    w = inputs.ADJOINT_256
    dt = torch.float64 if precision == mbo.F64 else torch.float32
    # target: projection of a heat-smoothed (tau = 1e-2) N(0,1) field, made on the GPU
    G = torch.tensor(inputs.normal_field(w.n, w.grid, inputs.ADJOINT_TARGET_SEED), dtype=dt, device="cuda")
    with mbo.Plan(w.grid, w.n, inputs.ADJOINT_TARGET_TAU, precision=precision) as pt:
        Td = pt.project(pt.diffuse(G))
    A0 = torch.tensor(w.field(), dtype=dt, device="cuda")
    plan = mbo.Plan(w.grid, w.n, w.tau, precision=precision)
    fw, bw = [], []
    for k in range(reps + 1):
        A = A0.clone().requires_grad_(True)
        tau = torch.tensor(w.tau, dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        AK = unrolled_mbo(A, tau, plan, w.iters, inputs.ADJOINT_CHECKPOINT)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss = 0.5 * ((AK - Td) ** 2).sum()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if k:  # the first run captures the graphs
            fw.append(t1 - t0)
            bw.append(t2 - t1)
    plan.close()
    f, b = min(fw), min(bw)
    return {"workload": "n3_256x256_K50_checkpoint10", "forward_ms": 1000 * f, "backward_ms": 1000 * b,
            "backward_over_forward": b / f,
            "point_steps_per_s": w.points * w.iters * 2 / (f + b)}


def run_batched(precision, autotune, steps):
    """64 fields of mixed n, grid and tau (seed 3), 50 iterations each, one graph:
    total point-iterations per second over all fields."""
    import torch
    from paper_1711_01365_amd import inputs, mbo
    bw = inputs.BatchedWorkload()
    dt = torch.float64 if precision == mbo.F64 else torch.float32
    t0 = time.perf_counter()
    bp = mbo.BatchedPlan([(m.grid, m.n, m.tau) for m in bw.members], precision=precision,
                         autotune=autotune)
    plan_s = time.perf_counter() - t0
    F0 = bp.pack([torch.tensor(m.field(), dtype=dt, device="cuda") for m in bw.members])
    F = F0.clone()
    F.copy_(F0)
    bp.iterate(F, bw.iters, logs=False)  # captures the graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        F.copy_(F0)
        bp.iterate(F, bw.iters, logs=False)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    bp.close()
    return {"workload": "64 fields seed 3, n in {2,3,4}, 128^2..1024^2, 50 it",
            "value": bw.points * bw.iters * steps / sec, "unit": "point-iterations/s",
            "ms_per_run": 1000.0 * sec / steps, "plan_s": plan_s, "autotune": bool(autotune)}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, runs=3, iters=20, iters_1t=3):
    """The FP64 oracle on the host's cores: the median of `runs` runs of the
    first `iters` iterations of the same workload with every OpenMP thread, and
    one run of `iters_1t` iterations on one thread (about 15 s in all)."""
    import oracle
    A0 = w.field()
    oracle.iterate(A0, w.tau, 1)  # builds and loads the library, warms the pages
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        oracle.iterate(A0, w.tau, iters)
        times.append(time.perf_counter() - t0)
    sec = sorted(times)[len(times) // 2]
    threads = oracle.num_threads()
    one = None
    if iters_1t > 0:
        oracle.set_num_threads(1)
        t0 = time.perf_counter()
        oracle.iterate(A0, w.tau, iters_1t)
        one = w.points * iters_1t / (time.perf_counter() - t0)
        oracle.set_num_threads(threads)
    return {
        "value": w.points * iters / sec,
        "unit": "point-iterations/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "median of %d runs of the first %d of the %d iterations of the same 512x512 n=3 workload, "
                  "FP64 C oracle on %d threads (%.2f s each); one thread: %d iterations"
                  % (runs, iters, w.iters, threads, sec, iters_1t),
        "value_1_thread": one,
        "cpu_model": cpu_model(),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the legs reported beside the main line (2048^2 control, 3-D, "
                         "batched, volume-preserving, paper examples, relaxed flows, sphere, "
                         "volume-preserving sphere, adjoint)")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--legs", default="control,3d,batched,volume,examples,relaxed,adjoint",
                    help="legs beside the main line (comma list of control, 3d, batched, volume, "
                         "examples, relaxed, adjoint, sphere)")
    ap.add_argument("--volume-only", action="store_true",
                    help="only the volume-preserving legs (for profiling them)")
    ap.add_argument("--peanut", action="store_true",
                    help="also run the peanut of Section 6.3 (133 M samples; about a minute of host set-up)")
    ap.add_argument("--surface-only", action="store_true",
                    help="only the sphere legs, float surfaces (for profiling them)")
    ap.add_argument("--only-3d", action="store_true", help="only the 3-D leg (for profiling it)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(a large field would be slab-decomposed by rows, with an all-to-all "
              "transpose each way per iteration); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    from paper_1711_01365_amd import inputs, mbo
    if args.volume_only:
        for wv in (inputs.VOLUME_HAAR_512, inputs.VOLUME_STAR_1024):
            r = run_volume(wv, args.steps, args.warmup)
            log("volume-preserving %s: %.3e point-iter/s, %.1f us/iteration (plain %.1f us)"
                % (wv.name, r["value"], r["us_per_iteration"], r["plain_mbo_us_per_iteration"]))
        return
    if args.only_3d:
        r = run_3d(args.steps, args.warmup)
        log("3-D %s: %.3e point-iter/s, row pass %.2f us (%.0f GB/s), plane pass %.2f us (%.0f GB/s)"
            % (r["workload"], r["value"], r["row_us"], r["row_GBps"], r["plane_us"], r["plane_GBps"]))
        return
    if args.surface_only:
        r = run_surface(args.steps, (("f32_f64fallback", mbo.F32_F64FALLBACK),))["f32_f64fallback"]
        log("sphere %s: %.3e sample-steps/s, %.1f us/step, diffuse %.1f us, m=%d grid=%d^3"
            % (r["workload"], r["value"], r["us_per_step"], r["diffuse_us"], r["samples"], r["grid"]))
        r = run_surface_volume(args.steps)
        log("volume-preserving sphere %s: %.3e sample-steps/s, %.1f us/step, m=%d, volume %d -> %d"
            % (r["workload"], r["value"], r["us_per_step"], r["samples"], r["volume_target"], r["volume_end"]))
        if args.peanut:
            r = run_peanut(args.steps)
            log("peanut %s: %.3e sample-steps/s, %.1f us/step, m=%d, grid=%d^3, set-up %.1f s, flips %s"
                % (r["workload"], r["value"], r["us_per_step"], r["samples"], r["grid"], r["setup_s"],
                   r["flips_first_steps"]))
        return
    w = inputs.HAAR_512
    log("workload %s: n=%d grid=%s tau=%g iterations=%d" % (w.name, w.n, w.grid, w.tau, w.iters))
    main_run = run_gpu(w, mbo.F32_F64FALLBACK, args.steps, args.warmup, timing_steps=3)
    log("fp32+fp64 fallback: %.3e point-iter/s, %.3f ms/step, row pass %.2f us, heat pass %.2f us"
        % (main_run["value"], main_run["ms_per_step"], main_run["row_us"], main_run["heat_us"]))
    f64 = None
    if not args.no_f64:
        f64 = run_gpu(w, mbo.F64, args.steps, min(args.warmup, 1), timing_steps=3)
        log("fp64: %.3e point-iter/s, row pass %.2f us, heat pass %.2f us"
            % (f64["value"], f64["row_us"], f64["heat_us"]))

    bytes_per_launch = 2 * w.n * w.n * 4 * w.points  # one read + one write of the FP32 field
    dominant_us = max(main_run["row_us"], main_run["heat_us"])
    dominant = "row_pass" if main_run["row_us"] >= main_run["heat_us"] else "heat_pass"
    banded = main_run["path"]["kind"] != "generic"
    kernel_name = {("row_pass", True): "row_fast<float, 3, 9, false>", ("row_pass", False): "row_pass<float, 3, 9, 0>",
                   ("heat_pass", True): "heat_fast<float, 9, TX>",
                   ("heat_pass", False): "col_pass<float, 2, 9>"}[(dominant, banded)]
    achieved = bytes_per_launch / (dominant_us * 1e-6) / 1e9
    traffic = read_traffic() if dominant == "row_pass" else None
    # what the band-limited row pass moves: the kept modes of the five packed
    # planes of every row, read and written (8 B each), and the det signs
    pl = (w.n * w.n + 1) // 2
    moved = 2 * pl * w.grid[0] * main_run["path"]["stored_modes"] * 8 + 2 * w.points
    out = {
        "metric": "MBO point-iterations/s (n=3, 512², FP32 vs FP64) + % of HBM peak",
        "value": main_run["value"],
        "unit": "point-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: Haar-random O(3) field per point, seed 1",
        "config": {"workload": "n3_512x512_haar_tau2e-4_200it_f32_f64fallback", "n": 3,
                   "grid": [512, 512], "tau": 2e-4, "iterations": 200,
                   "precision": "f32 + f64 fallback (sigma_min < 1e-3)"},
        "roofline": {"bound": "hbm", "kernel": kernel_name, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "bytes_per_launch": bytes_per_launch,
                     "avg_launch_us": dominant_us,
                     "moved_bytes_per_launch_model": moved if banded else bytes_per_launch},
        "path": main_run["path"],
        "kernels_us": {"row_pass": main_run["row_us"], "heat_pass": main_run["heat_us"]},
        "fallback_points_total": main_run["fallbacks_total"],
        "launch_shape": main_run["launch_shape"],
    }
    if f64 is not None:
        out["f64"] = {"value": f64["value"], "ms_per_step": f64["ms_per_step"],
                      "kernels_us": {"row_pass": f64["row_us"], "heat_pass": f64["heat_us"]},
                      "f32_over_f64": main_run["value"] / f64["value"]}
    legs = set() if args.no_extra else set(x.strip() for x in args.legs.split(",") if x.strip())
    if "control" in legs:
        out["control_2048"] = run_control_2048()
        log("2048^2 control: %.3e point-iter/s, row %.1f us (%.0f GB/s), heat %.1f us (%.0f GB/s)"
            % (out["control_2048"]["value"], out["control_2048"]["row_us"], out["control_2048"]["row_GBps"],
               out["control_2048"]["heat_us"], out["control_2048"]["heat_GBps"]))
    if "3d" in legs:
        out["config_3d"] = r = run_3d(3, 1)
        log("3-D n=3 128^3 fp32+fallback: %.3e point-iter/s, row pass %.2f us (%.0f GB/s), plane pass "
            "%.2f us (%.0f GB/s)" % (r["value"], r["row_us"], r["row_GBps"], r["plane_us"], r["plane_GBps"]))
    if "batched" in legs:
        out["batched"] = {"f32_autotuned": run_batched(mbo.F32, True, 3),
                          "f32_fixed_rules": run_batched(mbo.F32, False, 3),
                          "f64_autotuned": run_batched(mbo.F64, True, 2)}
        log("batched 64 fields: f32 tuned %.3e, f32 rules %.3e, f64 tuned %.3e point-iter/s"
            % (out["batched"]["f32_autotuned"]["value"], out["batched"]["f32_fixed_rules"]["value"],
               out["batched"]["f64_autotuned"]["value"]))
    if "volume" in legs:
        out["volume_preserving"] = {"n3_512x512_haar": run_volume(inputs.VOLUME_HAAR_512, 3, 1),
                                    "n2_1024x1024_star": run_volume(inputs.VOLUME_STAR_1024, 3, 1)}
        for k, r in out["volume_preserving"].items():
            log("volume-preserving %s: %.3e point-iter/s, %.1f us/iteration (plain %.1f us)"
                % (k, r["value"], r["us_per_iteration"], r["plain_mbo_us_per_iteration"]))
    if "examples" in legs:
        out["paper_examples"] = run_examples(3)
        for k, r in out["paper_examples"].items():
            log("paper example %s: %.3e point-iter/s, %.1f us/iteration, end: %d SO(2) points, index %s"
                % (k, r["value"], r["us_per_iteration"], r["so2_points_end"], r["index_end"]))
    if "relaxed" in legs:
        out["relaxed_flows"] = run_relaxed(3)
        for k, r in out["relaxed_flows"].items():
            log("relaxed flow %s: %.3e point-steps/s, %.1f us/step, E %.4g -> %.4g"
                % (k, r["value"], r["us_per_step"], r["energy_first_last"][0], r["energy_first_last"][1]))
    if "sphere" in legs:
        out["sphere"] = run_surface(1)
        for k, r in out["sphere"].items():
            log("sphere %s: %.3e sample-steps/s, %.1f us/step, diffuse %.1f us, m=%d grid=%d^3, SO-(3) %s"
                % (k, r["value"], r["us_per_step"], r["diffuse_us"], r["samples"], r["grid"],
                   r["so3minus_samples_first_last"]))
        out["sphere_volume_preserving"] = run_surface_volume(1)
        r = out["sphere_volume_preserving"]
        log("volume-preserving sphere: %.3e sample-steps/s, %.1f us/step, m=%d, volume %d -> %d"
            % (r["value"], r["us_per_step"], r["samples"], r["volume_target"], r["volume_end"]))
        if args.peanut:
            out["peanut"] = run_peanut(1)
            r = out["peanut"]
            log("peanut: %.3e sample-steps/s, %.1f us/step, m=%d, set-up %.1f s"
                % (r["value"], r["us_per_step"], r["samples"], r["setup_s"]))
    if "adjoint" in legs:
        out["adjoint"] = {"f32_f64fallback": run_adjoint(mbo.F32_F64FALLBACK, 2),
                          "f64": run_adjoint(mbo.F64, 2)}
        log("adjoint K=50 256^2: fp32+fb fwd %.1f ms bwd %.1f ms, fp64 fwd %.1f ms bwd %.1f ms"
            % (out["adjoint"]["f32_f64fallback"]["forward_ms"], out["adjoint"]["f32_f64fallback"]["backward_ms"],
               out["adjoint"]["f64"]["forward_ms"], out["adjoint"]["f64"]["backward_ms"]))
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w)
        log("cpu baseline: %.3e point-iter/s on %d threads" % (out["cpu_baseline"]["value"],
                                                             out["cpu_baseline"]["cores"]))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
