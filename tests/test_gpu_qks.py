"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the
general quasi-spherical grid of App. A (r0 = 0.4, h0 = 0.3): loading, initial
data, push, fused pass, field stages, full steps, diagnostics, the
single-precision form against FP64 and the adjoint against the reference
gradient.  Same bars as tests/test_gpu_parity.py."""
import math

import numpy as np
import pytest

from test_gpu_parity import (G, _sorted_state, assert_fields, assert_particles, assert_wald,  # noqa: F401
                             down, pair, up, wl)

pytestmark = pytest.mark.gpu

QKS = dict(r0=0.4, h0=0.3)


def test_qks_rejects_maps_outside_the_domain(G):
    """r0 must lie below r_min and h0 in (-1/2, 1) (where the polar map is
    increasing)."""
    w = wl("c1_64", 32)
    with pytest.raises(G.GrpicError):
        G.Context(w.a, w.M, w.r_min, w.r_max, 32, 32, r0=w.r_min)
    with pytest.raises(G.GrpicError):
        G.Context(w.a, w.M, w.r_min, w.r_max, 32, 32, h0=1.0)


def test_qks_loading(O, G):
    """Plasma loading (positions bit-exact, momenta to round-off) and test
    geodesics placed through the inverse of the polar map."""
    w = wl("c1_64", 48)
    prm, ctx = pair(O, G, w, **QKS)
    Po = O.particles_init(prm, 5000, 0, w.T, 0, w.seed)
    Pg = ctx.new_particles(len(Po["tag"]))
    ctx.particles_init(Pg, 5000, 0, w.T, 0, w.seed)
    Pg = down(Pg)
    for k in ("i1", "i2", "dx1", "dx2", "tag"):
        np.testing.assert_array_equal(Pg[k], Po[k], err_msg=k)
    assert_particles(prm, Po, Pg, tol=1e-13, what="qks init")
    w2 = wl("c2_512", 64)
    prm2, ctx2 = pair(O, G, w2, **QKS)
    Po = O.particles_init(prm2, 100, 0, 1.0, 500, 3)
    Pg = ctx2.new_particles(len(Po["tag"]))
    ctx2.particles_init(Pg, 100, 0, 1.0, 500, 3)
    assert_particles(prm2, Po, down(Pg), tol=1e-12, what="qks geodesic init")


def test_qks_initial_data(O, G):
    """Wald data (D pointwise, B by the discrete curl of the potential) and
    the monopole data on the general map."""
    w = wl("c1_64", 48)
    prm, ctx = pair(O, G, w, **QKS)
    Fo = O.fields_init_wald(prm, w.B0)
    Fg = ctx.new_fields()
    ctx.fields_init_wald(Fg, w.B0)
    assert_wald(O, prm, w.B0, Fo, Fg.cpu().numpy(), what="qks wald")
    wm = wl("c6_monopole", 48, n_absorb=6)
    prm, ctx = pair(O, G, wm, **QKS)
    Fo = O.fields_init_monopole(prm, wm.B0)
    Fg = ctx.new_fields()
    ctx.fields_init_monopole(Fg, wm.B0)
    assert_fields(Fo, Fg.cpu().numpy(), range(0, 33), what="qks monopole")


@pytest.mark.parametrize("h0", [0.3, -0.3])
def test_qks_push_per_step(O, G, h0):
    """Five push steps (frozen Wald field), each from the oracle's state, with
    particles next to both axes and photons among them (points concentrated
    toward the equator, h0 = 0.3, and toward the axes, h0 = -0.3)."""
    w = wl("c1_64", 48)
    prm, ctx = pair(O, G, w, r0=QKS["r0"], h0=h0)
    F = O.fields_init_wald(prm, w.B0)
    P = O.particles_init(prm, 8000, 0, w.T, 0, w.seed)
    P["i2"][:40] = 0
    P["dx2"][:40] = np.linspace(1e-6, 0.3, 40)
    P["i2"][40:80] = 47
    P["dx2"][40:80] = np.linspace(0.7, 1 - 1e-6, 40)
    P["tag"][80::9] = 7
    for k in ("i2", "dx2"):
        P[k + "p"][:] = P[k]
    Fg = up({"F": F})["F"]
    for step in range(5):
        Pg = up(P)
        O.push(prm, F, P)
        ctx.push(Fg, Pg)
        assert_particles(prm, P, down(Pg), what=f"qks push {step}")


def test_qks_field_advance(O, G):
    """Both field stages from a perturbed Wald state with currents, 2 filter
    passes and an absorbing layer."""
    w = wl("c1_64", 48)
    prm, ctx = pair(O, G, w, charge_scale=0.05, n_filter=2, n_absorb=6, **QKS)
    F = O.fields_init_wald(prm, w.B0)
    g = np.random.default_rng(0)
    F[:12] *= 1 + 0.1 * g.normal(size=F[:12].shape)
    F[18:24] = 0.01 * g.normal(size=F[18:24].shape)
    for stage in (0, 1):
        Fg = up({"F": F})["F"]
        O.field_advance(prm, F, stage)
        ctx.field_advance(Fg, stage)
        assert_fields(F, Fg.cpu().numpy(), range(0, 24), what=f"qks stage {stage}")


@pytest.mark.parametrize("fused", [False, True])
def test_qks_full_step(O, G, fused):
    """Full PIC steps with charge, filter passes and the absorbing layer on
    the general map (the C5 recipe on a 48^2 grid)."""
    w = wl("c5_4096", 48, n_absorb=6)
    prm, ctx = pair(O, G, w, charge_scale=0.02, **QKS)
    if fused:
        F, P = _sorted_state(O, prm, w, ppc=8)
    else:
        F = O.fields_init_wald(prm, w.B0)
        P = O.particles_init(prm, 8000, 0, w.T, 0, w.seed)
    for step in range(4):
        Fg, Pg = up({"F": F})["F"], up(P)
        O.step(prm, F, P)
        ctx.step(Fg, Pg, fused=fused)
        assert_fields(F, Fg.cpu().numpy(), list(range(0, 24)), what=f"qks step {step}")
        assert_particles(prm, P, down(Pg), what=f"qks step {step}", prev=not fused)


def test_qks_diagnostics(O, G):
    """E, L at the time-centred positions and the Gauss residual."""
    w = wl("c1_64", 48)
    prm, ctx = pair(O, G, w, charge_scale=0.03, n_filter=2, **QKS)
    F = O.fields_init_wald(prm, w.B0)
    P = O.particles_init(prm, 5000, 0, w.T, 0, w.seed)
    for _ in range(3):
        O.step(prm, F, P)
    Fg, Pg = up({"F": F})["F"], up(P)
    d = ctx.diagnostics(Fg, Pg, w.B0, per_particle=True, gauss_plane=True)
    E, L = O.energy_momentum(prm, P, w.B0)
    live = P["tag"] != 0
    np.testing.assert_allclose(d["E"].cpu().numpy()[live], E[live], rtol=1e-12)
    np.testing.assert_allclose(d["L"].cpu().numpy()[live], L[live], rtol=1e-12, atol=1e-12)
    res, mx, scale = O.gauss_residual(prm, F, P)
    assert d["gauss_scale"] == pytest.approx(scale, rel=1e-12)
    assert np.abs(d["gauss_res"].cpu().numpy() - res).max() <= 1e-12 * scale


def test_qks_fp32_against_fp64(G):
    """The single-precision form on the general map: one push of a loaded
    plasma against the FP64 push of the same (rounded) state."""
    import torch
    w = wl("c3_2048", 128)
    kw = dict(cfl=w.cfl, n_iter=w.n_iter, small_angle=w.small_angle, **QKS)
    c32 = G.Context(w.a, w.M, w.r_min, w.r_max, w.n_r, w.n_th, precision=G.GRPIC_FP32, **kw)
    c64 = G.Context(w.a, w.M, w.r_min, w.r_max, w.n_r, w.n_th, dt=c32.dt, **kw)
    n = w.n_particles
    P32 = c32.new_particles(n)
    c32.particles_init(P32, 0, w.ppc, w.T, 0, w.seed)
    F32 = c32.new_fields()
    c32.fields_init_wald(F32, w.B0)
    P64 = {k: (v.to(torch.float64) if v.dtype == torch.float32 else v.clone())
           for k, v in P32.items()}
    F64 = F32[:33].double()
    c32.push(F32, P32)
    c64.push(F64, P64)
    torch.cuda.synchronize()
    a = {k: v.cpu().numpy() for k, v in P32.items()}
    b = {k: v.cpu().numpy() for k, v in P64.items()}
    assert ((a["tag"] != 0) != (b["tag"] != 0)).sum() == 0
    live = b["tag"] != 0
    for d in ("1", "2"):
        xa = a["i" + d] + a["dx" + d].astype(np.float64)
        xb = b["i" + d] + b["dx" + d]
        assert np.abs(xa - xb)[live].max() <= 2e-6
    for k in ("u1", "u2", "u3"):
        e = np.abs(a[k].astype(np.float64) - b[k])[live]
        sc = np.abs(b[k])[live] + np.abs(b[k])[live].max() * 1e-3
        assert np.median(e / sc) <= 1e-6 and (e / sc).max() <= 1e-4, k


def test_qks_adjoint_matches_reference_gradient(O, G):
    """The adjoint of the frozen-field push on the general map against
    autograd of the oracle restatement (24^2, 10 steps, checkpoints every 5)."""
    import torch
    import oracle.adjoint as A
    from paper_2511_17701_amd.adjoint import FrozenFieldPush, FrozenRun
    from paper_2511_17701_amd.workloads import WORKLOADS
    w = WORKLOADS["c4_256"].scaled(24, 24)
    ctx = G.Context(w.a, w.M, w.r_min, w.r_max, 24, 24, cfl=w.cfl, n_iter=w.n_iter,
                    small_angle=w.small_angle, **QKS)
    F1 = ctx.new_fields()
    ctx.fields_init_wald(F1, 1.0)
    P = ctx.new_particles(800)
    ctx.particles_init(P, 400, 0, w.T, 0, 7)
    P["tag"][::7] = 3
    P["tag"][3::11] = 7
    torch.cuda.synchronize()
    steps = 10
    u0 = torch.stack([P["u1"], P["u2"], P["u3"]], 1).clone().requires_grad_(True)
    B0 = torch.tensor(w.B0, dtype=torch.float64, requires_grad=True)
    run = FrozenRun(ctx, P, steps, 5)
    out = FrozenFieldPush.apply(u0, B0, run)
    dxi = math.log((w.r_max - QKS["r0"]) / (w.r_min - QKS["r0"])) / 24
    loss = (out[:, 2] / (dxi * (w.r_min - QKS["r0"]) * torch.exp(out[:, 0] * dxi))).mean()
    loss.backward()
    prm = O.Params.make(w.a, w.M, w.r_min, w.r_max, 24, 24, ctx.dt, n_iter=w.n_iter, **QKS)
    st = A.state_from({k: v.cpu().numpy() for k, v in P.items()})
    F1o = torch.from_numpy(O.fields_init_wald(prm, 1.0))
    loss_o, gu_o, gB0_o, _ = A.gradients(prm, F1o, w.B0, st, steps)
    assert abs(loss.item() - loss_o) <= 1e-12 * abs(loss_o)
    g, go = u0.grad.cpu().numpy(), gu_o.numpy()
    err = np.abs(g - go).max(axis=1) / (np.abs(go).max(axis=1) + 1e-300)
    print(f"\n[qks adjoint vs reference] per-particle rel err median {np.median(err):.3g} "
          f"p99 {np.quantile(err, 0.99):.3g}; dL/dB0 {B0.grad.item():.12g} vs {gB0_o:.12g}")
    assert np.quantile(err, 0.99) <= 1e-9
    assert abs(B0.grad.item() - gB0_o) <= 1e-9 * abs(gB0_o)


@pytest.mark.parametrize("n", [96, 768])
def test_qks_push_fine_grids(O, G, n):
    """The push and the fused pass on the general map at finer grids (96^2
    and 768^2: in-cell angle steps up to 0.05 and 0.007 rad); three push
    steps and a fused step from the oracle's state, with particles next to
    both axes."""
    w = wl("c1_64", n)
    prm, ctx = pair(O, G, w, charge_scale=0.3, **QKS)
    F = O.fields_init_wald(prm, w.B0)
    P = O.particles_init(prm, 15000, 0, w.T, 0, w.seed)
    P["i2"][:60] = np.arange(60) % 3
    P["dx2"][:60] = np.linspace(1e-6, 0.99, 60)
    P["i2"][60:120] = n - 1 - np.arange(60) % 3
    P["dx2"][60:120] = np.linspace(0.01, 1 - 1e-6, 60)
    P["tag"][120::13] = 7
    for k in ("i2", "dx2"):
        P[k + "p"][:] = P[k]
    Fg = up({"F": F})["F"]
    for step in range(3):
        Pg = up(P)
        O.push(prm, F, P)
        ctx.push(Fg, Pg)
        assert_particles(prm, P, down(Pg), what=f"qks fine push n={n} step {step}")
    Fg, Pg = up({"F": F})["F"], up(P)
    O.push(prm, F, P)
    O.deposit(prm, F, P)
    ctx.push_deposit(Fg, Pg)
    assert_particles(prm, P, down(Pg), what=f"qks fine fused n={n}", prev=False)
    Jg = Fg.cpu().numpy()
    if n > 96:
        # at 768^2 the particles placed in the first cells sit a few 1e-4 rad
        # from an axis, where J^3 ~ 1/sin^2(theta) at the path midpoint turns
        # the last bit of the midpoint into ~1e-12 of the plane's maximum:
        # compare the nodes more than 3 cells from either axis to the plane
        # bar, the rest to 1e-11
        g = prm.ng
        inner = (slice(None), slice(g + 3, g + n - 2))
        for c in range(18, 21):
            sc = np.abs(F[c]).max()
            assert np.abs(F[c][inner] - Jg[c][inner]).max() <= 1e-12 * sc, c
            assert np.abs(F[c] - Jg[c]).max() <= 1e-11 * sc, c
    else:
        assert_fields(F, Jg, range(18, 21), what=f"qks fine J n={n}")


def test_qks_fp32_full_steps(G):
    """The single-precision form on the general map over 100 full PIC steps
    of the C3 recipe (a = 0.99, B0 = 10, 32 ppc) at 256^2, against the FP64
    form from the same rounded state: the bars of the standard grid's test."""
    import torch
    from test_gpu_fp32 import compare
    w = wl("c3_2048", 256)
    kw = dict(cfl=w.cfl, n_iter=w.n_iter, small_angle=w.small_angle, charge_scale=w.charge_scale,
              n_filter=w.n_filter, n_absorb=w.n_absorb, **QKS)
    c32 = G.Context(w.a, w.M, w.r_min, w.r_max, w.n_r, w.n_th, precision=G.GRPIC_FP32, **kw)
    c64 = G.Context(w.a, w.M, w.r_min, w.r_max, w.n_r, w.n_th, dt=c32.dt, **kw)
    P32 = c32.new_particles(w.n_particles)
    c32.particles_init(P32, 0, w.ppc, w.T, 0, w.seed)
    F32 = c32.new_fields()
    c32.fields_init_wald(F32, w.B0)
    P64 = {k: (v.to(torch.float64) if v.dtype == torch.float32 else v.clone())
           for k, v in P32.items()}
    F64 = F32[:33].double()
    for _ in range(w.steps):
        c32.step(F32, P32, fused=True)
        c64.step(F64, P64, fused=True)
    torch.cuda.synchronize()
    st, live = compare(w, P32, P64, f"qks {w.steps} full steps")
    d32 = c32.diagnostics(F32, P32, w.B0, per_particle=True)
    d64 = c64.diagnostics(F64, P64, w.B0, per_particle=True)
    E32 = d32["E"].double().cpu().numpy()[live]
    E64 = d64["E"].cpu().numpy()[live]
    e_err = np.abs(E32 - E64) / np.maximum(np.abs(E64), 1.0)
    g = 2
    inner = (slice(None), slice(g + 2, g + w.n_th - 1))
    err_in, err_all = [], []
    for c in range(6):
        a = F32[c].double().cpu().numpy()
        b = F64[c].cpu().numpy()
        s = np.abs(b).max()
        err_all.append(np.abs(a - b).max() / s)
        err_in.append(np.abs(a - b)[inner].max() / s)
    print(f"[qks fp32 vs fp64] energy p99 {np.quantile(e_err, 0.99):.3g}; D, B inner "
          f"{max(err_in):.3g}, all {max(err_all):.3g}")
    assert d32["n_nonfinite"] == 0 and d64["n_nonfinite"] == 0
    assert st["tag_mismatch"] <= max(2, 1e-5 * st["n"])
    assert st["u_p99"] <= 1e-5
    assert st["u_med"] <= 2e-6
    assert np.quantile(e_err, 0.99) <= 1e-5
    assert max(err_in) <= 1e-5
    assert max(err_all) <= 1e-4
