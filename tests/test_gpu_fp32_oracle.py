"""The single-precision form against the FP64 CPU oracle, through the C ABI.

The oracle starts from the GPU's FP32 state and fields widened to FP64 (the
same numbers), so the comparison measures what one FP32 step adds:
  - one fused push + deposit pass (C3 recipe, a = 0.99, 32 ppc, 256^2 and
    512^2, the latter on the short-series kernel the benchmark times):
    per-particle momenta within 1e-5 of max(|u_i|, gamma c_i) (median within
    1e-6), positions within 3e-6 of a cell, currents per plane within 1e-5 of
    the plane's largest value;
  - the separate push (which also writes the previous position) to the same
    bars, and with the FP64 convergence test of the implicit iterations on
    (iter_tol > 0; the oracle runs its fixed count);
  - one full PIC step with 4 filter passes and the absorbing layer (C5 recipe
    at 128^2 and 32^2): D, B, J per plane within 1e-5 of their largest value;
  - the benchmark's workload at full size (C5, 4096^2, 2.68e8 particles) in
    the benchmark's launch configuration: 20,000 sampled slots after one
    fused pass, to the particle bars above.
Momenta scales c_i are the code-unit scales dr/dx1, r dth, r sin(theta).
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_17701_amd import grpic
    torch.cuda.set_device(0)
    return grpic


def setup(O, G, name, n, charge_scale, iter_tol=0.0, n_absorb=None):
    from paper_2511_17701_amd.workloads import WORKLOADS
    w = WORKLOADS[name].scaled(n, n)
    na = w.n_absorb if n_absorb is None else n_absorb
    c32 = G.Context(w.a, w.M, w.r_min, w.r_max, n, n, cfl=w.cfl, n_iter=w.n_iter,
                    small_angle=w.small_angle, charge_scale=charge_scale, n_filter=w.n_filter,
                    n_absorb=na, iter_tol=iter_tol, precision=G.GRPIC_FP32)
    prm = O.Params.make(w.a, w.M, w.r_min, w.r_max, n, n, c32.dt, n_iter=w.n_iter,
                        small_angle=w.small_angle, charge_scale=charge_scale,
                        n_filter=w.n_filter, n_absorb=na)
    P32 = c32.new_particles(w.n_particles)
    c32.particles_init(P32, 0, w.ppc, w.T, 0, w.seed)
    F32 = c32.new_fields()
    c32.fields_init_wald(F32, w.B0)
    Po = {k: (v.cpu().numpy().astype(np.float64) if v.is_floating_point() else v.cpu().numpy())
          for k, v in P32.items()}
    Fo = F32[:33].double().cpu().numpy().copy()
    return w, prm, c32, P32, F32, Po, Fo


def particle_errors(w, Pg, Po):
    a = {k: v.cpu().numpy() for k, v in Pg.items()}
    np.testing.assert_array_equal(a["tag"], Po["tag"])
    live = Po["tag"] != 0
    dxi = math.log(w.r_max / w.r_min) / w.n_r
    dth = math.pi / w.n_th
    x_err = np.zeros(live.sum())
    for d in ("1", "2"):
        xa = a["i" + d] + a["dx" + d].astype(np.float64)
        xo = Po["i" + d] + Po["dx" + d]
        x_err = np.maximum(x_err, np.abs(xa - xo)[live])
    r = w.r_min * np.exp((Po["i1"] + Po["dx1"]) * dxi)
    th = (Po["i2"] + Po["dx2"]) * dth
    c = [dxi * r, r * dth, r * np.maximum(np.abs(np.sin(th)), 1e-5)]
    gam = np.sqrt(1 + sum((Po[k] / ci) ** 2 for k, ci in zip(("u1", "u2", "u3"), c)))
    u_err = np.zeros(live.sum())
    for k, ci in zip(("u1", "u2", "u3"), c):
        e = np.abs(a[k].astype(np.float64) - Po[k]) / np.maximum(np.abs(Po[k]), gam * ci)
        u_err = np.maximum(u_err, e[live])
    return x_err, u_err


def plane_errors(Fg, Fo, planes):
    out = []
    for c in planes:
        a = Fg[c].double().cpu().numpy()
        s = np.abs(Fo[c]).max()
        out.append(float(np.abs(a - Fo[c]).max() / s) if s > 0 else float(np.abs(a).max()))
    return out


def report(what, x_err, u_err, planes=None):
    msg = (f"\n[fp32 vs oracle] {what}: x max {x_err.max():.3g} cells, u median "
           f"{np.median(u_err):.3g} p99 {np.quantile(u_err, 0.99):.3g} max {u_err.max():.3g}")
    if planes is not None:
        msg += f"; planes {np.array(planes)}"
    print(msg)


@pytest.mark.parametrize("n", [256, 512])
def test_fp32_fused_pass_against_oracle(O, G, n):
    """At 512^2 (dtheta small enough) the pass runs the short-series kernel
    that the benchmark times, currents included."""
    w, prm, c, Pg, Fg, Po, Fo = setup(O, G, "c3_2048", n, charge_scale=1e-3)
    c.push_deposit(Fg, Pg)
    O.push(prm, Fo, Po)
    O.deposit(prm, Fo, Po)
    x_err, u_err = particle_errors(w, Pg, Po)
    jerr = plane_errors(Fg, Fo, [18, 19, 20])
    report(f"fused pass {n}^2", x_err, u_err, jerr)
    assert x_err.max() <= 3e-6
    assert u_err.max() <= 1e-5 and np.median(u_err) <= 1e-6
    assert max(jerr) <= 1e-5


@pytest.mark.parametrize("iter_tol", [0.0, 1e-7])
def test_fp32_push_against_oracle(O, G, iter_tol):
    """The separate push, with and without the FP64 convergence test; the
    previous position it writes is the start of the step exactly."""
    w, prm, c, Pg, Fg, Po, Fo = setup(O, G, "c3_2048", 256, charge_scale=1e-3, iter_tol=iter_tol)
    start = {k: Po[k].copy() for k in ("i1", "i2", "dx1", "dx2")}
    c.push(Fg, Pg)
    O.push(prm, Fo, Po)
    x_err, u_err = particle_errors(w, Pg, Po)
    report(f"push (iter_tol {iter_tol:g})", x_err, u_err)
    for k in ("i1", "i2", "dx1", "dx2"):
        got = Pg[k + "p"].cpu().numpy()
        np.testing.assert_array_equal(got.astype(start[k].dtype), start[k], err_msg=k + "p")
    assert x_err.max() <= 3e-6
    assert u_err.max() <= 1e-5 and np.median(u_err) <= 1e-6


@pytest.mark.parametrize("n", [128, 32, 512])
def test_fp32_full_step_against_oracle(O, G, n):
    """One full PIC step with 4 filter passes and an 8-cell absorbing layer
    (C5 recipe, kappa = 1e-3): fields and particles.  At 32^2 the current
    filter takes its path for planes with fewer rows than a strip stages; at
    512^2 the push runs the short-series kernel the benchmark times."""
    w, prm, c, Pg, Fg, Po, Fo = setup(O, G, "c5_4096", n, charge_scale=1e-3, n_absorb=8)
    c.step(Fg, Pg)
    O.step(prm, Fo, Po)
    x_err, u_err = particle_errors(w, Pg, Po)
    ferr = plane_errors(Fg, Fo, list(range(6)) + [18, 19, 20])
    report("full step", x_err, u_err, ferr)
    assert x_err.max() <= 3e-6
    assert u_err.max() <= 1e-5 and np.median(u_err) <= 1e-6
    assert max(ferr) <= 1e-5


def test_c5_fp32_fused_launch_sampled(O, G):
    """The benchmark's workload at full size (C5: 4096^2, 16 ppc = 2.68e8
    particles, FP32) in the launch configuration the benchmark times (the
    single-precision series kernel of fine grids): after one fused push +
    deposit pass, a sample of 20,000 slots matches the oracle's push of the
    same pre-push states (widened to FP64) in the same widened fields, to the
    bars of the 256^2 case."""
    import torch
    from paper_2511_17701_amd.workloads import WORKLOADS
    w = WORKLOADS["c5_4096"]
    c = G.Context(w.a, w.M, w.r_min, w.r_max, w.n_r, w.n_th, cfl=w.cfl, n_iter=w.n_iter,
                  small_angle=w.small_angle, charge_scale=w.charge_scale, n_filter=w.n_filter,
                  n_absorb=w.n_absorb, precision=G.GRPIC_FP32)
    prm = O.Params.make(w.a, w.M, w.r_min, w.r_max, w.n_r, w.n_th, c.dt, n_iter=w.n_iter,
                        small_angle=w.small_angle, charge_scale=w.charge_scale,
                        n_filter=w.n_filter, n_absorb=w.n_absorb)
    n = w.n_particles
    Pg = c.new_particles(n)
    c.particles_init(Pg, 0, w.ppc, w.T, 0, w.seed)
    Fg = c.new_fields()
    c.fields_init_wald(Fg, w.B0)
    idx = np.sort(np.random.default_rng(3).choice(n, 20000, replace=False))
    it = torch.from_numpy(idx).cuda()
    S = {k: v.index_select(0, it).cpu().numpy() for k, v in Pg.items()}
    So = {k: (v.astype(np.float64) if v.dtype.kind == "f" else v) for k, v in S.items()}
    Fo = Fg[:33].double().cpu().numpy()
    c.push_deposit(Fg, Pg)
    torch.cuda.synchronize()
    O.push(prm, Fo, So)
    Pd = {k: v.index_select(0, it) for k, v in Pg.items()}
    x_err, u_err = particle_errors(w, Pd, So)
    # cells whose inner edge lies below r = 3M take the FP64 metric in the push
    dxi = math.log(w.r_max / w.r_min) / w.n_r
    i_fp64 = math.ceil(math.log(3.0 * w.M / w.r_min) / dxi)
    report(f"c5 full size, fused launch, 20000 sampled slots ({int((S['i1'] < i_fp64).sum())} "
           f"in FP64-metric cells)", x_err, u_err)
    assert x_err.max() <= 3e-6
    assert u_err.max() <= 1e-5 and np.median(u_err) <= 1e-6
    del Pg, Fg, Fo
    torch.cuda.empty_cache()
