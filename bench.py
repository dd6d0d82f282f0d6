"""Benchmark of the GRPIC hot path on one MI355X.

One step = one full PIC step of the paper's loop (Sec. 3.4): pre-push field
stage, push (gather + EM/geodesic update + coordinate update), charge-
conserving deposit, post-deposit field stage.  Inputs (Wald field, Maxwell-
Juttner plasma) are generated on the device before timing.  Prints one JSON
line; see the design doc for the roofline accounting.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, GB/s
FP64_VECTOR_TFLOPS = 78.6    # MI355X FP64 vector peak

# Algorithmic HBM bytes per particle of the FP64 push: reads tag (1), i1 i2 (8),
# dx1 dx2 (16), u1 u2 u3 (24), phi (8) = 57 B; writes i1p i2p dx1p dx2p (24),
# i1 i2 dx1 dx2 (24), u (24), phi (8), tag (1) = 81 B.
PUSH_BYTES_FP64 = 57 + 81
# Deposit: reads tag (1), w (8), previous and current cell + offset (48),
# u (24) = 81 B per particle; currents are accumulated in cache.
DEPOSIT_BYTES_FP64 = 81


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2_512")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default=None,
                    help="storage precision (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--iter-tol", type=float, default=0.0,
                    help="FP64 convergence test of the implicit iterations (0: fixed count)")
    ap.add_argument("--unfused", action="store_true",
                    help="separate push and deposit passes (default: one fused pass)")
    ap.add_argument("--sort-every", type=int, default=10,
                    help="cell-sort the particles every k steps (0: never)")
    return ap.parse_args()


def cpu_baseline(w, dt):
    """The oracle (FP64 C, OpenMP over particles) timed on the host cores on
    a bounded sample: `cpu_steps` full steps of the same workload."""
    import numpy as np  # noqa: F401
    import oracle as O
    prm = O.Params.make(w.a, w.M, w.r_min, w.r_max, w.n_r, w.n_th, dt, n_iter=w.n_iter,
                        small_angle=w.small_angle, charge_scale=w.charge_scale,
                        n_filter=w.n_filter, n_absorb=w.n_absorb)
    F = O.fields_init_wald(prm, w.B0)
    P = O.particles_init(prm, w.n_pairs_total if w.ppc == 0 else 0, w.ppc, w.T, w.n_geo, w.seed)
    n = int((P["tag"] != 0).sum())
    steps = ARGS.cpu_steps
    t0 = time.perf_counter()
    for _ in range(steps):
        if w.full_step:
            O.step(prm, F, P)
        else:
            O.push(prm, F, P)
            O.deposit(prm, F, P)
    t = time.perf_counter() - t0
    return {"value": n * steps / t, "unit": "particle pushes/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"{steps} full steps of the {w.name} workload (all {n} particles, "
                      f"{w.n_r}x{w.n_th} grid), {t:.1f} s"}


def main():
    global ARGS
    ARGS = parse()
    if ARGS.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_2511_17701_amd import grpic
    from paper_2511_17701_amd.workloads import WORKLOADS

    w = WORKLOADS[ARGS.workload]
    precision = ARGS.precision or w.precision
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    ctx = grpic.Context(w.a, w.M, w.r_min, w.r_max, w.n_r, w.n_th, cfl=w.cfl, n_iter=w.n_iter,
                        small_angle=w.small_angle, charge_scale=w.charge_scale,
                        n_filter=w.n_filter, n_absorb=w.n_absorb, iter_tol=ARGS.iter_tol,
                        precision=grpic.GRPIC_FP32 if precision == "fp32" else grpic.GRPIC_FP64)
    F = ctx.new_fields(dev)
    ctx.fields_init_wald(F, w.B0)
    P = ctx.new_particles(w.n_particles, dev)
    ctx.particles_init(P, w.n_pairs_total if w.ppc == 0 else 0, w.ppc, w.T, w.n_geo, w.seed)
    Q = ctx.new_particles(w.n_particles, dev) if ARGS.sort_every > 0 else None
    state = {"P": P, "Q": Q, "n": 0}
    torch.cuda.synchronize()
    d0 = ctx.diagnostics(F, P, w.B0)
    live0 = sum(d0["n_alive"])

    def step(ev=None):
        P = state["P"]
        if w.full_step:
            ctx.field_advance(F, grpic.PRE_PUSH)
        if ev is not None:
            ev[0].record()
        if ARGS.unfused:
            ctx.push(F, P)
        else:
            ctx.push_deposit(F, P)
        if ev is not None:
            ev[1].record()
        if ARGS.unfused:
            ctx.deposit(P, F)
        if ev is not None:
            ev[2].record()
        if w.full_step:
            ctx.field_advance(F, grpic.POST_DEPOSIT)
        state["n"] += 1
        if ARGS.sort_every > 0 and state["n"] % ARGS.sort_every == 0:
            ctx.sort(state["P"], state["Q"])
            state["P"], state["Q"] = state["Q"], state["P"]

    for _ in range(ARGS.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(ARGS.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record()
    for k in range(ARGS.steps):
        step(evs[k])
    t_end.record()
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    push_ms = sum(e[0].elapsed_time(e[1]) for e in evs) / ARGS.steps
    dep_ms = sum(e[1].elapsed_time(e[2]) for e in evs) / ARGS.steps
    P = state["P"]
    d1 = ctx.diagnostics(F, P, w.B0)
    live1 = sum(d1["n_alive"])
    assert d1["n_nonfinite"] == 0, "non-finite particles after the run"
    live = 0.5 * (live0 + live1)
    ms = total_ms / ARGS.steps
    value = live / (ms * 1e-3)
    push_gbs = PUSH_BYTES_FP64 * live / (push_ms * 1e-3) / 1e9
    out = {
        "metric": "particle pushes/s (gather+push+deposit)",
        "value": value,
        "unit": "particle pushes/s",
        "n_gpus": 1,
        "steps": ARGS.steps,
        "warmup": ARGS.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32 (FP64 horizon metric)",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": f"{w.n_r}x{w.n_th}", "a": w.a,
                   "r_range": [w.r_min, w.r_max], "particles": w.n_particles, "ppc": w.ppc,
                   "test_geodesics": w.n_geo, "T": w.T, "B0": w.B0, "n_iter": w.n_iter,
                   "dt": ctx.dt, "full_step": w.full_step, "precision": precision,
                   "charge_scale": w.charge_scale,
                   "sort_every": ARGS.sort_every, "iter_tol": ARGS.iter_tol},
        "roofline": {"bound": "hbm", "kernel": "push_kernel", "achieved": push_gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": push_gbs / HBM_PEAK_GBS,
                     "traffic": None,
                     "bytes_per_particle": PUSH_BYTES_FP64, "avg_launch_ms": push_ms},
        "kernels_ms_per_step": {"push" if ARGS.unfused else "push_deposit": push_ms,
                                "deposit": dep_ms,
                                "fields_and_rest": ms - push_ms - dep_ms},
        "push_deposit_rate": live / ((push_ms + dep_ms) * 1e-3),
        "live_particles": [live0, live1],
    }
    if not ARGS.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, ctx.dt)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
