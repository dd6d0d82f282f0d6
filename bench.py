"""Benchmark of the GRPIC hot path on one MI355X.

One step = one full PIC step of the paper's loop (Sec. 3.4): pre-push field
stage, push + charge-conserving deposit (one fused pass, grpic_push_deposit),
post-deposit field stage; the particles are cell-sorted every --sort-every
steps (inside the timed region).  Inputs (Wald field, Maxwell-Juttner
plasma) are generated on the device before timing.  Prints one JSON line.

Roofline of the dominant kernel (the fused push+deposit pass): FP64 (or, in
the single-precision form, FP32 + FP64) vector FLOPs per particle counted by
rocprofv3 for this kernel on this workload (FMA = 2; the figures and the
command that measured them are in profiles/), times the particles of one
launch, over the launch time measured here with HIP events on the launch
stream; peak = 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP x 2.4 GHz = 78.6 TFLOP/s
(FP64 vector; also the non-packed FP32 rate, packed FP32 being disabled).
`traffic` = HBM bytes per launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE
summary of the same kernel scaled by the copy-kernel calibration, or null if
the kernel sources changed since (the summary records their hash).

--copy-calibration runs a plain device copy of known size (for the
FETCH_SIZE / WRITE_SIZE calibration) and exits.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_VECTOR_TFLOPS = 78.6    # MI355X FP64 vector (= non-packed FP32 vector)
HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per particle of the fused pass (FP64): reads tag (1),
# i1 i2 (8), dx1 dx2 (16), u (24), w (8), phi (8) = 65; writes i dx (24),
# u (24), phi (8), tag (1) = 57.  FP32 form: 4-byte reals: reads
# 1 + 8 + 8 + 12 + 4 + 4 = 37, writes 16 + 12 + 4 + 1 = 33.
FUSED_BYTES = {"fp64": 65 + 57, "fp32": 37 + 33}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's step count)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c5_4096")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default=None,
                    help="storage precision (default: the workload's)")
    ap.add_argument("--unfused", action="store_true",
                    help="separate push and deposit passes (default: one fused pass)")
    ap.add_argument("--sort-every", type=int, default=10,
                    help="cell-sort the particles every k steps (0: never)")
    ap.add_argument("--sort-rank", choices=["auto", "fused", "separate"], default="auto",
                    help="the sort's rank pass in the fused pass of the sort step (grpic_push_deposit_ranked) "
                         "or as a kernel of its own; auto: fused in FP64, separate in FP32 (the faster of the "
                         "two in each form at 4096^2 and 2048^2)")
    ap.add_argument("--iter-tol", type=float, default=0.0,
                    help="FP64 convergence test of the implicit iterations (0: fixed count)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="oracle steps of the CPU baseline (0: 8, or 2 above 2^23 particles)")
    ap.add_argument("--cpu-single-pairs", type=int, default=1 << 15,
                    help="pairs of the single-thread oracle figure (0: skip it)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the timing of the other precision form and of the adjoint")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="time only the differentiation form (the adjoint leg) and exit")
    ap.add_argument("--copy-calibration", action="store_true")
    return ap.parse_args()


def source_hash():
    """Hash of the sources of the fused push + deposit kernels (particles.hpp,
    geometry.hpp) with comments and blank space removed: a counter summary of
    that kernel stays valid across comment-only edits and changes elsewhere."""
    import re
    h = hashlib.sha256()
    files = [os.path.join(ROOT, "paper_2511_17701_amd", "csrc", f) for f in ("geometry.hpp", "particles.hpp")]
    for f in files:
        with open(f, encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        text = " ".join(text.split())
        h.update(os.path.basename(f).encode() + b"\0" + text.encode())
    return h.hexdigest()[:16]


class HipEvents:
    """HIP timing events recorded on torch's current stream, created with
    hipEventDisableSystemFence: a record then neither writes back nor
    invalidates the caches, so timing a kernel does not slow the work around
    it (the host reads results only after a device synchronisation)."""

    DISABLE_SYSTEM_FENCE = 0x20000000

    def __init__(self):
        import ctypes
        import torch
        # the HIP runtime torch (and libgrpic) already use in this process
        path = next(line.split()[-1] for line in open("/proc/self/maps") if "libamdhip64" in line)
        self.c = ctypes
        self.lib = ctypes.CDLL(path)
        self.torch = torch

    def _check(self, rc, what):
        if rc != 0:
            raise RuntimeError(f"{what} failed with HIP error {rc}")

    def create(self):
        ev = self.c.c_void_p()
        self._check(self.lib.hipEventCreateWithFlags(self.c.byref(ev), self.c.c_uint(self.DISABLE_SYSTEM_FENCE)),
                    "hipEventCreateWithFlags")
        return ev

    def record(self, ev):
        stream = self.c.c_void_p(self.torch.cuda.current_stream().cuda_stream)
        self._check(self.lib.hipEventRecord(ev, stream), "hipEventRecord")

    def elapsed(self, a, b):
        ms = self.c.c_float()
        self._check(self.lib.hipEventElapsedTime(self.c.byref(ms), a, b), "hipEventElapsedTime")
        return ms.value

    def destroy(self, ev):
        self._check(self.lib.hipEventDestroy(ev), "hipEventDestroy")


def profile_figures(name):
    """key: value lines of a committed profile summary (empty if absent)."""
    path = os.path.join(ROOT, "profiles", name)
    out = {}
    if os.path.exists(path):
        with open(path) as fh:
            for line in fh:
                if ":" in line and not line.startswith((" ", "#")):
                    k, v = line.split(":", 1)
                    out[k.strip()] = v.strip()
    return out


def cpu_model():
    """The host CPU's model name and logical CPU count (as /proc/cpuinfo states them)."""
    model, n = "unknown", 0
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    n += 1
    except OSError:
        pass
    return model, n


def cpu_baseline(w, dt):
    """The oracle (FP64 C, OpenMP over particles) timed on the host cores on a
    bounded sample of the workload.

    Grids up to 2^20 cells: `cpu_steps` full PIC steps (8) of the whole
    particle set (2^22 pairs in uniformly drawn cells above 2^23 particles).
    Larger grids: the oracle's field stages alone take minutes per step there
    (its field loops are serial), so the sample is the metric's own work,
    gather + push + deposit, of 2^21 pairs in uniformly drawn cells for
    `cpu_steps` steps (2) in the workload's initial fields.  A second figure
    runs the same sample kind on one thread with `cpu_single_pairs` pairs."""
    import oracle as O
    prm = O.Params.make(w.a, w.M, w.r_min, w.r_max, w.n_r, w.n_th, dt, n_iter=w.n_iter,
                        small_angle=w.small_angle, charge_scale=w.charge_scale,
                        n_filter=w.n_filter, n_absorb=w.n_absorb, r0=w.r0, h0=w.h0)
    F = O.fields_init_monopole(prm, w.B0) if w.init == "monopole" else O.fields_init_wald(prm, w.B0)
    big_grid = w.n_r * w.n_th > 2 ** 20
    full = w.full_step and not big_grid

    def sample(n_pairs, steps, threads):
        if n_pairs is None:
            P = O.particles_init(prm, w.n_pairs_total if w.ppc == 0 else 0, w.ppc, w.T, w.n_geo,
                                 w.seed)
        else:
            P = O.particles_init(prm, n_pairs, 0, w.T, w.n_geo, w.seed)
        n = int((P["tag"] != 0).sum())
        Fs = F.copy()
        O.set_num_threads(threads)
        used = O.num_threads()
        t0 = time.perf_counter()
        for _ in range(steps):
            if full:
                O.step(prm, Fs, P)
            else:
                O.push(prm, Fs, P)
                O.deposit(prm, Fs, P)
        return n * steps / (time.perf_counter() - t0), n, time.perf_counter() - t0, used

    host_threads = O.num_threads()
    if big_grid:
        n_pairs, steps = 2 ** 21, ARGS.cpu_steps or 2
    elif w.n_particles > 2 ** 23:
        n_pairs, steps = 2 ** 22, ARGS.cpu_steps or 2
    else:
        n_pairs, steps = None, ARGS.cpu_steps or 8
    value, n, t, used = sample(n_pairs, steps, host_threads)
    kind = "full FP64 PIC steps" if full else "FP64 gather + push + deposit passes (no field stages)"
    what = f"{n} particles ({'all' if n_pairs is None else f'{n_pairs} pairs in uniformly drawn cells'})"
    model, logical = cpu_model()
    out = {"value": value, "unit": "particle pushes/s", "cores": used, "kind": "oracle",
           "sample": f"{steps} {kind} of the {w.name} workload ({w.n_r}x{w.n_th} grid, {what}), "
                     f"{t:.1f} s",
           "cpu_model": model, "host_logical_cpus": logical}
    if ARGS.cpu_single_pairs > 0:
        v1, n1, t1, _ = sample(ARGS.cpu_single_pairs, 1, 1)
        out["single_thread"] = {"value": v1, "unit": "particle pushes/s", "cores": 1,
                                "sample": f"1 {'full FP64 PIC step' if full else 'FP64 gather + push + deposit pass'}"
                                          f" of {n1} particles in uniformly drawn cells, {t1:.1f} s"}
    O.set_num_threads(host_threads)
    return out


def copy_calibration():
    import torch
    n = 1 << 27                                  # 2^27 doubles = 1 GiB
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "launches": 3}))


def rank_in_pass(precision):
    """Whether the sort step's fused pass also does the sort's rank pass."""
    return ARGS.sort_rank == "fused" or (ARGS.sort_rank == "auto" and precision == "fp64")


class Run:
    """A context, a field set and a particle set of a workload in one form."""

    def __init__(self, grpic, w, precision, dev):
        import torch
        self.G, self.w, self.precision = grpic, w, precision
        self.ctx = grpic.Context(w.a, w.M, w.r_min, w.r_max, w.n_r, w.n_th, cfl=w.cfl,
                                 n_iter=w.n_iter, small_angle=w.small_angle,
                                 charge_scale=w.charge_scale, n_filter=w.n_filter,
                                 n_absorb=w.n_absorb, iter_tol=ARGS.iter_tol, r0=w.r0, h0=w.h0,
                                 precision=grpic.GRPIC_FP32 if precision == "fp32"
                                 else grpic.GRPIC_FP64)
        self.F = self.ctx.new_fields(dev)
        if w.init == "monopole":
            self.ctx.fields_init_monopole(self.F, w.B0)
        else:
            self.ctx.fields_init_wald(self.F, w.B0)
        self.P = self.ctx.new_particles(w.n_particles, dev)
        self.ctx.particles_init(self.P, w.n_pairs_total if w.ppc == 0 else 0, w.ppc, w.T,
                                w.n_geo, w.seed)
        self.Q = self.ctx.new_particles(w.n_particles, dev) if ARGS.sort_every > 0 else None
        self.n = 0
        torch.cuda.synchronize()

    def step(self, ev=None):
        """One step; on a sort step the fused pass also ranks the slots for
        the sort (grpic_push_deposit_ranked, then grpic_sort_ranked).
        Returns whether the fused pass ranked."""
        ctx, F, P, w = self.ctx, self.F, self.P, self.w
        sort_now = ARGS.sort_every > 0 and (self.n + 1) % ARGS.sort_every == 0
        ranked = sort_now and not ARGS.unfused and rank_in_pass(self.precision)
        if w.full_step:
            ctx.field_advance(F, self.G.PRE_PUSH)
        if ev is not None:
            ev[0]()
        if ARGS.unfused:
            ctx.push(F, P)
        else:
            ctx.push_deposit(F, P, ranked=ranked)
        if ev is not None:
            ev[1]()
        if ARGS.unfused:
            ctx.deposit(P, F)
            if ev is not None:
                ev[2]()
        if w.full_step:
            ctx.field_advance(F, self.G.POST_DEPOSIT)
        self.n += 1
        if sort_now:
            ctx.sort(self.P, self.Q, ranked=ranked)
            self.P, self.Q = self.Q, self.P
        return ranked

    def timed(self, steps, warmup):
        """Average ms per step, per-step kernel times (HIP events on the
        launch stream) and live particle counts before / after."""
        import torch
        live0 = sum(self.ctx.diagnostics(self.F, self.P, self.w.B0)["n_alive"])
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        he = HipEvents()
        evs = [[he.create() for _ in range(3 if ARGS.unfused else 2)] for _ in range(steps)]
        for e in evs:
            if not ARGS.unfused:
                e.append(e[1])  # no second kernel: the deposit interval is empty
        t0, t1 = he.create(), he.create()
        torch.cuda.synchronize()
        he.record(t0)
        ranked = [self.step([lambda e=e: he.record(e) for e in evs[k]]) for k in range(steps)]
        he.record(t1)
        torch.cuda.synchronize()
        total = he.elapsed(t0, t1)
        t_pass = [he.elapsed(e[0], e[1]) for e in evs]
        # the fused pass of the steps without the rank pass (the kernel the
        # roofline and the profiles describe), the ranked one separately
        plain = [t for t, r in zip(t_pass, ranked) if not r] or t_pass
        self.k1_all = sum(t_pass) / steps
        self.k1_ranked = (sum(t for t, r in zip(t_pass, ranked) if r) / sum(ranked)) if any(ranked) else None
        k1 = sum(plain) / len(plain)
        k2 = sum(he.elapsed(e[1], e[2]) for e in evs) / steps if ARGS.unfused else 0.0
        for e in evs:
            for x in e[:3 if ARGS.unfused else 2]:
                he.destroy(x)
        he.destroy(t0)
        he.destroy(t1)
        d1 = self.ctx.diagnostics(self.F, self.P, self.w.B0)
        assert d1["n_nonfinite"] == 0, "non-finite particles after the run"
        return total / steps, k1, k2, live0, sum(d1["n_alive"])


def adjoint_leg(grpic, dev):
    """The differentiation form on its workload (C4: 256^2, a = 0.9, 10^6
    particles, frozen Wald field, 50 push steps, checkpoints every 10): the
    forward pass (grpic_push) and the adjoint sweep (the replay of each
    segment plus one grpic_push_adjoint per step) timed with HIP events on the
    launch stream, and the adjoint kernel alone."""
    import torch
    from paper_2511_17701_amd.adjoint import FrozenFieldPush, FrozenRun
    from paper_2511_17701_amd.workloads import WORKLOADS
    w = WORKLOADS["c4_256"]
    ctx = grpic.Context(w.a, w.M, w.r_min, w.r_max, w.n_r, w.n_th, cfl=w.cfl, n_iter=w.n_iter,
                        small_angle=w.small_angle)
    P = ctx.new_particles(2 * w.n_pairs, dev)
    ctx.particles_init(P, w.n_pairs, 0, w.T, 0, w.seed)
    run = FrozenRun(ctx, P, w.steps, 10)
    he = HipEvents()
    ev = [he.create() for _ in range(3)]
    u0 = torch.stack([P["u1"], P["u2"], P["u3"]], 1).clone().requires_grad_(True)
    B0 = torch.tensor(w.B0, dtype=torch.float64, requires_grad=True)
    torch.cuda.synchronize()
    he.record(ev[0])
    out = FrozenFieldPush.apply(u0, B0, run)
    he.record(ev[1])
    out[:, 2].mean().backward()
    he.record(ev[2])
    torch.cuda.synchronize()
    fwd, bwd = he.elapsed(ev[0], ev[1]), he.elapsed(ev[1], ev[2])
    # the adjoint kernel alone, 10 launches from the final state
    F = run.fields(w.B0)
    n = P["tag"].numel()
    g = torch.ones((5, n), dtype=torch.float64, device=dev)
    gB = torch.zeros(n, dtype=torch.float64, device=dev)
    ctx.push_adjoint(F, w.B0, P, g, g, gB)
    torch.cuda.synchronize()
    he.record(ev[0])
    for _ in range(10):
        ctx.push_adjoint(F, w.B0, P, g, g, gB)
    he.record(ev[1])
    torch.cuda.synchronize()
    k_ms = he.elapsed(ev[0], ev[1]) / 10
    for e in ev:
        he.destroy(e)
    return {"workload": w.name, "particles": n, "steps": w.steps, "checkpoint_every": 10,
            "forward_ms": fwd, "backward_ms": bwd,
            "gradient_particle_steps_per_s": n * w.steps / ((fwd + bwd) * 1e-3),
            "adjoint_kernel_ms": k_ms, "adjoint_particles_per_s": n / (k_ms * 1e-3),
            "accuracy": "tests/test_gpu_adjoint.py: adjoint against the oracle's reference gradient "
                        "and against central differences on the full C4 workload"}


def main():
    global ARGS
    ARGS = parse()
    if ARGS.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; run with --gpus 1"}))
        sys.exit(2)
    if ARGS.copy_calibration:
        copy_calibration()
        return
    import torch
    from paper_2511_17701_amd import grpic
    from paper_2511_17701_amd.workloads import WORKLOADS

    if ARGS.adjoint_only:
        torch.cuda.set_device(0)
        print(json.dumps({"differentiation": adjoint_leg(grpic, torch.device("cuda:0"))}), flush=True)
        return
    w = WORKLOADS[ARGS.workload]
    if ARGS.steps is None:
        ARGS.steps = w.steps
    precision = ARGS.precision or w.precision
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    run = Run(grpic, w, precision, dev)
    ms, k1, k2, live0, live1 = run.timed(ARGS.steps, ARGS.warmup)
    dt = run.ctx.dt
    live = 0.5 * (live0 + live1)
    value = live / (ms * 1e-3)
    kname = "push" if ARGS.unfused else "push_deposit"

    figs = profile_figures(f"{kname}_{w.name}_{precision}_pmc.txt")
    current = figs.get("source_sha256") == source_hash()
    flops_pp = float(figs["flops_per_particle"]) if current and "flops_per_particle" in figs else None
    lanes = float(figs["valu_active_lane_fraction"]) if current and "valu_active_lane_fraction" in figs else None
    executed = flops_pp * live / (k1 * 1e-3) / 1e12 if flops_pp else None
    # the method's own FLOPs: the counted lane slots times the fraction of lanes
    # active in the kernel's VALU instructions (masked-off lanes do no work)
    achieved = executed * lanes if executed and lanes else executed
    traffic = None
    if current and "hbm_bytes_per_particle" in figs:
        traffic = float(figs["hbm_bytes_per_particle"]) * live
    gbs = FUSED_BYTES[precision] * live / (k1 * 1e-3) / 1e9
    roofline = {
        "bound": "alu", "kernel": f"{kname}_kernel", "achieved": achieved,
        "peak": PEAK_VECTOR_TFLOPS, "unit": "TFLOP/s",
        "frac": achieved / PEAK_VECTOR_TFLOPS if achieved else None,
        "traffic": traffic, "avg_launch_ms": k1, "particles_per_launch": live,
        "flops_per_particle": flops_pp,
        "frac_basis": ("FLOPs: the kernel's counted FP32/FP64 VALU lane slots (wave instructions x 64, "
                       "FMA = 2) times the measured fraction of active lanes "
                       f"({lanes:.3f})" if lanes else
                       "FLOPs: the kernel's counted FP32/FP64 VALU lane slots (wave instructions x 64, "
                       "FMA = 2), lanes masked off in divergent iterations included"),
        "achieved_executed_lane_slots": executed,
        "peak_basis": "256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz: FP64 and non-packed FP32 "
                      "vector issue (packed FP32, the chip's 157.3 TFLOP/s, is not used by this code)",
    }
    if current and "valu_instructions_per_particle" in figs:
        # a wave64 VALU instruction occupies its SIMD (16 lanes) for 4 cycles
        vi = float(figs["valu_instructions_per_particle"])
        cycles = vi * live / 64.0 * 4.0
        roofline["valu_issue"] = {"instructions_per_particle": vi,
                                  "frac_of_issue_cycles": cycles / (1024 * 2.4e9 * k1 * 1e-3)}
    if not ARGS.unfused:
        roofline["hbm_view"] = {"algorithmic_bytes_per_particle": FUSED_BYTES[precision],
                                "GB_per_s": gbs, "frac_of_8TBs": gbs / HBM_PEAK_GBS}
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
        "dtype": "f64" if precision == "fp64" else "f32 (+f64 horizon metric)",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": f"{w.n_r}x{w.n_th}", "a": w.a,
                   "r_range": [w.r_min, w.r_max], "map_r0_h0": [w.r0, w.h0],
                   "particles": w.n_particles, "ppc": w.ppc,
                   "test_geodesics": w.n_geo, "T": w.T, "B0": w.B0, "n_iter": w.n_iter,
                   "dt": dt, "full_step": w.full_step, "n_filter": w.n_filter,
                   "n_absorb": w.n_absorb, "precision": precision,
                   "charge_scale": w.charge_scale,
                   "pass": "unfused" if ARGS.unfused else "fused",
                   "sort_every": ARGS.sort_every,
                   "sort_rank": "in the fused pass" if not ARGS.unfused and rank_in_pass(precision)
                   else "separate pass",
                   "iter_tol": ARGS.iter_tol},
        "roofline": roofline,
        "kernels_ms_per_step": {kname: k1, **({"deposit": k2} if ARGS.unfused else {}),
                                **({"push_deposit_ranked (sort steps)": run.k1_ranked}
                                   if run.k1_ranked is not None else {}),
                                "fields_sort_rest": ms - run.k1_all - k2},
        "live_particles": [live0, live1],
    }
    if not ARGS.no_forms:
        other = "fp32" if precision == "fp64" else "fp64"
        del run
        torch.cuda.empty_cache()
        r2 = Run(grpic, w, other, dev)
        ms2, k12, _, a0, a1 = r2.timed(ARGS.steps, ARGS.warmup)
        t64, t32 = (ms, ms2) if precision == "fp64" else (ms2, ms)
        out["precision_forms"] = {
            other: {"ms_per_step": ms2, "value": 0.5 * (a0 + a1) / (ms2 * 1e-3),
                    f"{kname}_ms": k12},
            "fp32_speedup_over_fp64": t64 / t32,
            "fp32_accuracy": "tests/test_gpu_fullsize.py: C3 at 2048^2, 100 full steps against "
                             "the FP64 form, every particle above 1e-5 attributed; C5 Gauss drift "
                             "over 200 steps at 4096^2 <= 1e-6; tests/test_gpu_fp32_oracle.py: "
                             "one step against the oracle",
        }
        del r2
        torch.cuda.empty_cache()
        out["precision_forms"]["differentiation"] = adjoint_leg(grpic, dev)
        torch.cuda.empty_cache()
    if not ARGS.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, dt)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
