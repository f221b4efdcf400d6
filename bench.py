#!/usr/bin/env python3
"""Benchmark of the hot path: one step = one full gradient evaluation
(fwi_gradient: forward sweep with checkpoints, residual and misfit, adjoint
sweep with re-forward of each checkpoint segment, gradient imaging) for all
shots of the workload, with inputs resident in device memory.

Metric: forward + adjoint Gcell-updates/s = NX * NY * nt * shots * 2 / time,
NX x NY the total grid including the CPML.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload large|survey|tiny]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2506_20513_amd import inputs as I  # noqa: E402
from paper_2506_20513_amd import rocprof_summary  # noqa: E402

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, AMD public specification

WORKLOADS = {"large": I.config_large, "survey": I.config_survey, "tiny": I.config_tiny}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Per-step algorithmic bytes of each stencil kernel for one cell and all its
# shots: a forward cell-update reads and writes Ez, Hx, Hy (24 B); the
# adjoint one reads and writes the three adjoint fields and reads the forward
# Ez^n (28 B); Ca and Cs (8 B per cell) are shared by all shots.  One launch
# advances several time levels; a gradient runs nt forward-sweep levels,
# nt segment re-forward levels (the same forward step, recomputed from the
# checkpoints) and nt adjoint levels.
PER_CELL_UPDATE = {"k_fwd_sweep": 24.0, "k_fwd_reforward": 24.0, "k_adj": 28.0}


def algorithmic_bytes(kernel: str, cell_updates: float, shots: int) -> float:
    """Algorithmic bytes for `cell_updates` cell x shot x step updates."""
    return cell_updates * (PER_CELL_UPDATE[kernel] + 8.0 / shots)


def cpu_model() -> str:
    """The host CPU's model name (Linux), or the platform's processor."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(cfg, e0, s0, src, rec, w):
    """The FP64 oracle as it stands on the host cores: the whole gradient of
    one shot of the same workload over the full window (forward sweep with
    checkpoints, then each segment re-run forward and the adjoint run over
    it).  Its observed traces are zero (the residual is then the traces
    themselves), which costs the same as any other data."""
    import oracle
    P = oracle.Problem(e0, s0, cfg.npml, cfg.dx, cfg.dy, cfg.dt, cpml_order=cfg.cpml_order,
                       cpml_sigma_scale=cfg.cpml_sigma_scale, cpml_kappa_max=cfg.cpml_kappa_max,
                       cpml_alpha_max=cfg.cpml_alpha_max)
    obs0 = np.zeros((1, cfg.nt, cfg.nrec))
    t0 = time.perf_counter()
    P.gradient_checkpointed(src[:1], rec[:1], w[:1], obs0, cfg.nt)
    el = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cores = min(cores, os.cpu_count() or cores)
    return {"value": cfg.NX * cfg.NY * cfg.nt * 2 / el / 1e9, "unit": "Gcell-updates/s",
            "cores": cores, "kind": "oracle", "cpu": cpu_model(),
            "s_per_shot_gradient": round(el, 2),
            "sample": f"1 of {cfg.nshots} shots, all {cfg.nt} steps of the {cfg.NX}x{cfg.NY} "
                      f"grid: forward with checkpoints, segment re-forward and adjoint, "
                      f"gradient, FP64, {el:.1f} s"}


def bench_uneven(args):
    """Batched gradients of independent problems of uneven size (96 models,
    interior grids 200x100 .. 640x320, 1500-4000 steps, 8 shots x 64
    receivers): one plan, one graph replay per step."""
    import torch
    from paper_2506_20513_amd import fwi
    cfgs = I.config_uneven(args.models)
    dev = "cuda"
    keep, probs = [], []
    t0 = time.perf_counter()
    for cfg in cfgs:
        e, s, e0, s0 = I.model_for(cfg)
        src, rec = I.geometry(cfg)
        w = torch.from_numpy(I.wavelets(cfg)).to(dev)
        grid = fwi.grid_from_config(cfg)
        geom = fwi.Geometry(src, rec, w)
        et, st_, e0t, s0t = (torch.from_numpy(a).to(dev) for a in (e, s, e0, s0))
        obs = torch.empty((cfg.nshots, cfg.nt, cfg.nrec), device=dev)
        wsf = fwi.alloc_workspace(fwi.workspace_bytes(grid, geom, fwi.FWI_SAVE_NONE), dev)
        fwi.fdtd_forward(grid, geom, et, st_, obs, fwi.FWI_SAVE_NONE, wsf)
        mis = torch.empty(1, dtype=torch.float64, device=dev)
        ge = torch.empty((cfg.NY, cfg.NX), device=dev)
        gs = torch.empty((cfg.NY, cfg.NX), device=dev)
        probs.append(fwi.BatchProblem(grid, geom, e0t, s0t, obs, mis, ge, gs))
        keep.append((w, wsf))
    torch.cuda.synchronize()
    keep = [k[0] for k in keep]
    log(f"bench: {len(cfgs)} problems ready ({time.perf_counter() - t0:.1f} s)")
    ws_bytes = fwi.batch_workspace_bytes(probs)
    ws = fwi.alloc_workspace(ws_bytes, dev)
    t0 = time.perf_counter()
    plan = fwi.BatchPlan(probs, ws, autotune=not args.no_autotune)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    info = plan.info()
    log(f"bench: plan in {plan_s:.1f} s, workspace {ws_bytes / 1e9:.1f} GB, {info}")
    for k in range(args.warmup):
        plan.run()
        torch.cuda.synchronize()
        log(f"bench: warmup {k + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        plan.run()
        torch.cuda.synchronize()
        log(f"bench: step {k + 1}/{args.steps} done")
    el = time.perf_counter() - t0
    ms_per_step = el / args.steps * 1e3
    updates = sum(c.NX * c.NY * c.nt * c.nshots * 2 for c in cfgs)
    interior = sum(c.nx * c.ny * c.nt * c.nshots * 2 for c in cfgs)
    alg = sum(c.NX * c.NY * c.nt * (c.nshots * (24.0 + 28.0) + 16.0) for c in cfgs)
    out = {
        "metric": "Gcell-updates/s fwd+adjoint FDTD (eps_r/sigma gradient), batched uneven models",
        "value": round(updates / (ms_per_step / 1e3) / 1e9, 3),
        "unit": "Gcell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"uneven: {len(cfgs)} independent models, interior 200x100 .. "
                               f"640x320 at dx=0.01 m, 1500-4000 steps, 8 shots x 64 receivers, "
                               f"Ricker 200 MHz", "models": len(cfgs),
                   "workspace_GB": round(ws_bytes / 1e9, 2)},
        "interior_gcells": round(interior / (ms_per_step / 1e3) / 1e9, 3),
        "effective_hbm_frac": round(alg / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "plan": info, "plan_seconds": round(plan_s, 2),
    }
    if args.sequential:
        # the same problems one after another through fwi_gradient, in one
        # workspace large enough for any of them
        need = max(fwi.workspace_bytes(p.grid, p.geom, fwi.GRADIENT_WORKSPACE) for p in probs)
        del ws
        plan.close()
        torch.cuda.empty_cache()
        w1 = fwi.alloc_workspace(need, dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for p in probs:
            a = p.arrays
            fwi.fwi_gradient(p.grid, p.geom, a[0], a[1], a[2], a[3], a[4], a[5], None, w1)
        torch.cuda.synchronize()
        seq = time.perf_counter() - t0
        out["sequential_ms"] = round(seq * 1e3, 1)
        out["batched_speedup"] = round(seq * 1e3 / ms_per_step, 2)
        log(f"bench: sequential single-problem calls {seq:.2f} s")
    plan.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOADS) + ["uneven"])
    ap.add_argument("--models", type=int, default=96, help="uneven workload: number of models")
    ap.add_argument("--no-autotune", action="store_true", help="uneven workload: default bands")
    ap.add_argument("--sequential", action="store_true",
                    help="uneven workload: also time the problems one by one")
    ap.add_argument("--sample-every", type=int, default=32,
                    help="time every k-th launch of each hot kernel with HIP events")
    ap.add_argument("--nt", type=int, default=None,
                    help="override the number of time steps (short profiler runs)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB "
                         "(calibrates the profiler's HBM byte counters)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: this build runs on one "
              "GPU only (shots would shard across GPUs with one gradient all-reduce, "
              "which is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2506_20513_amd import fwi

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    fwi.lib()
    if args.workload == "uneven":
        return bench_uneven(args)

    cfg = WORKLOADS[args.workload]()
    if args.nt is not None:
        cfg = cfg.with_(nt=args.nt)
    dev = "cuda"
    if args.copy_probe_mb > 0:
        n = args.copy_probe_mb * (1 << 20) // 4
        a = torch.ones(n, device=dev)
        b = torch.empty(n, device=dev)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"bench: copy probe {args.copy_probe_mb} MiB done")
        del a, b
    log(f"bench: workload {cfg.name} NX={cfg.NX} NY={cfg.NY} nt={cfg.nt} shots={cfg.nshots} "
        f"receivers={cfg.nrec}")
    e, s, e0, s0 = I.model_for(cfg)
    src, rec = I.geometry(cfg)
    w = I.wavelets(cfg)
    grid = fwi.grid_from_config(cfg)
    wt = torch.from_numpy(w).to(dev)
    geom = fwi.Geometry(src, rec, wt)
    et, st_, e0t, s0t = (torch.from_numpy(a).to(dev) for a in (e, s, e0, s0))
    S, R, nt = cfg.nshots, cfg.nrec, cfg.nt

    # observed data: forward of the true model (input preparation, untimed)
    ws_fwd = fwi.alloc_workspace(fwi.workspace_bytes(grid, geom, fwi.FWI_SAVE_NONE), dev)
    obs = torch.empty((S, nt, R), device=dev)
    fwi.fdtd_forward(grid, geom, et, st_, obs, fwi.FWI_SAVE_NONE, ws_fwd)
    torch.cuda.synchronize()
    del ws_fwd
    log("bench: observed data ready")

    ws_bytes = fwi.workspace_bytes(grid, geom, fwi.GRADIENT_WORKSPACE)
    ws = fwi.alloc_workspace(ws_bytes, dev)
    K = fwi.checkpoint_interval(grid, geom)
    mis = torch.empty(1, dtype=torch.float64, device=dev)
    ge = torch.empty((cfg.NY, cfg.NX), device=dev)
    gs = torch.empty((cfg.NY, cfg.NX), device=dev)
    log(f"bench: workspace {ws_bytes / 1e9:.1f} GB, checkpoint interval {K}")

    for k in range(args.warmup):
        fwi.fwi_gradient(grid, geom, e0t, s0t, obs, mis, ge, gs, None, ws)
        torch.cuda.synchronize()
        log(f"bench: warmup {k + 1}/{args.warmup} done, misfit {mis.item():.6e}")

    kt = {}
    groups = 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        tm = fwi.fwi_timing(sample_every=args.sample_every)
        fwi.fwi_gradient_timed(grid, geom, e0t, s0t, obs, mis, ge, gs, None, ws, tm)
        groups = tm.shot_groups
        for name, v in tm.as_dict().items():
            a = kt.setdefault(name, {"launches": 0, "timed": 0, "ms": 0.0, "updates": 0.0})
            a["launches"] += v["launches"]
            a["timed"] += v["timed"]
            a["ms"] += v["avg_ms"] * v["timed"]
            a["updates"] += v["cell_updates"]
        log(f"bench: step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_per_step = el / args.steps * 1e3

    cells = cfg.NX * cfg.NY
    updates = cells * nt * S * 2
    value = updates / (ms_per_step / 1e3) / 1e9
    kernels = {}
    # each launch covers one shot group (the library runs the shots in
    # `groups` concurrent groups); the coefficient bytes are shared by the
    # shots of one launch
    shots_per_launch = S / groups
    for name, a in kt.items():
        if a["launches"] == 0:
            continue
        avg = a["ms"] / a["timed"] if a["timed"] else 0.0
        kb = algorithmic_bytes(name, a["updates"], shots_per_launch) / a["launches"]
        kernels[name] = {"launches_per_step": a["launches"] // args.steps,
                         "avg_ms": avg,
                         "ms_per_step": avg * a["launches"] / args.steps,
                         "bytes_per_launch": kb,
                         "algorithmic_GBps": kb / (avg / 1e3) / 1e9 if avg > 0 else None}
    # measured HBM bytes per launch of each kernel, from the committed
    # counter summary of these same kernel sources and workload (else None)
    counters = os.path.join(ROOT, "profiles", f"stencil_{args.workload}_counters.md")
    for name, kd in kernels.items():
        tb = rocprof_summary.read_traffic(counters, name, [cfg.NX, cfg.NY], S)
        kd["traffic_bytes_per_launch"] = tb
        kd["measured_GBps"] = tb / (kd["avg_ms"] / 1e3) / 1e9 if tb and kd["avg_ms"] else None
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    # mean number of stencil launches running at once over the timed steps
    in_flight = sum(k["ms_per_step"] for k in kernels.values()) / ms_per_step
    # measured HBM traffic of all stencil launches of a step over the step
    # time (null unless every kind has a counter figure)
    step_traffic = None
    if all(k["traffic_bytes_per_launch"] for k in kernels.values()):
        step_traffic = sum(k["traffic_bytes_per_launch"] * k["launches_per_step"]
                           for k in kernels.values())
    step_gbps = step_traffic / (ms_per_step / 1e3) / 1e9 if step_traffic else None
    by = kernels[dom]["bytes_per_launch"]
    achieved = kernels[dom]["algorithmic_GBps"]
    traffic = kernels[dom]["traffic_bytes_per_launch"]
    measured = kernels[dom]["measured_GBps"]
    # algorithmic bytes of the whole step (forward + adjoint, one pass each)
    alg_step = cells * nt * (S * (24.0 + 28.0) + 16.0)
    out = {
        "metric": "Gcell-updates/s fwd+adjoint FDTD (eps_r/sigma gradient)",
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.nx}x{cfg.ny} interior + {cfg.npml}-cell CPML "
                               f"({cfg.NX}x{cfg.NY}), dx={cfg.dx} m, {nt} steps, "
                               f"{S} shots x {R} receivers, Ricker {cfg.f0 / 1e6:.0f} MHz",
                   "grid": [cfg.NX, cfg.NY], "nt": nt, "shots": S, "receivers": R,
                   "checkpoint_interval": K, "workspace_GB": round(ws_bytes / 1e9, 2)},
        "s_per_shot_gradient": round(ms_per_step / 1e3 / S, 5),
        "interior_gcells": round(cfg.nx * cfg.ny * nt * S * 2 / (ms_per_step / 1e3) / 1e9, 3),
        "effective_hbm_frac": round(alg_step / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "traffic_unit": "bytes/launch",
                     "bytes_per_launch": by,
                     "measured_GBps": round(measured, 1) if measured else None,
                     "measured_frac": round(measured / HBM_PEAK_GBS, 4) if measured else None,
                     "shot_groups": groups,
                     "launches_in_flight": round(in_flight, 3),
                     "step_measured_GBps": round(step_gbps, 1) if step_gbps else None,
                     "step_measured_frac": round(step_gbps / HBM_PEAK_GBS, 4) if step_gbps else None,
                     "note": "achieved counts the algorithmic bytes of one HBM sweep per time "
                             "step; one launch advances several steps per sweep (temporal "
                             "blocking), so frac can exceed 1. measured_frac divides the "
                             "profiler's HBM bytes per launch (traffic) by the same duration. "
                             "The shots run in shot_groups concurrent groups on separate "
                             "streams; each launch covers one group, and its duration includes "
                             "the other groups' launches running beside it (launches_in_flight "
                             "on average), so per-launch rates are a share of the GPU's; "
                             "effective_hbm_frac is the whole step's algorithmic rate and "
                             "step_measured_frac its measured HBM traffic over the step."},
        "kernels": kernels,
        "misfit": float(mis.item()),
    }
    if not args.no_cpu_baseline:
        log(f"bench: cpu baseline (oracle, one shot, {nt} steps)")
        del ws
        torch.cuda.empty_cache()
        out["cpu_baseline"] = cpu_baseline(cfg, e0, s0, src, rec, w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
