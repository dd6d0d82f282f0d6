"""The single-precision form (int32 cell + FP32 offsets, momenta, fields and
currents; FP64 metric in the horizon region and FP64 iteration residual)
against the FP64 form of the same library, through the C ABI.

Loading and the Wald initial field are computed in FP64 and rounded once, so
the FP32 state must equal the rounded FP64 state bit for bit.  Dynamics are
compared from one common state (the FP32 state, widened for the FP64 run):
  - one push: positions and momenta per particle;
  - the deposit: currents per plane;
  - 100 full PIC steps of the single-precision workload (a = 0.99, 32
    particles per cell, B0 = 10) at a reduced grid: per-particle relative
    error of the momenta and the conserved energy, fields per plane, all
    within 1e-5;
  - the Gauss-law residual of the FP32 run, with current filtering and the
    absorbing layer, must not drift by more than 1e-6 of its largest term.
Momentum errors are relative to max(|u_i|, gamma c_i), c_i the code-unit
scale of component i (dr/dx1, r dth, r sin theta).
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


def wl(name, n, **kw):
    from paper_2511_17701_amd.workloads import WORKLOADS
    return WORKLOADS[name].scaled(n, n, **kw)


def contexts(G, w, charge_scale=None, n_filter=None, n_absorb=None):
    kw = dict(cfl=w.cfl, n_iter=w.n_iter, small_angle=w.small_angle,
              charge_scale=w.charge_scale if charge_scale is None else charge_scale,
              n_filter=w.n_filter if n_filter is None else n_filter,
              n_absorb=w.n_absorb if n_absorb is None else n_absorb)
    c32 = G.Context(w.a, w.M, w.r_min, w.r_max, w.n_r, w.n_th, precision=G.GRPIC_FP32, **kw)
    c64 = G.Context(w.a, w.M, w.r_min, w.r_max, w.n_r, w.n_th, dt=c32.dt, **kw)
    assert c64.dt == c32.dt
    return c32, c64


def widen(P):
    import torch
    return {k: (v.to(torch.float64) if v.dtype == torch.float32 else v.clone())
            for k, v in P.items()}


def host(P):
    return {k: v.cpu().numpy() for k, v in P.items()}


def u_scale(w, P):
    dxi = math.log(w.r_max / w.r_min) / w.n_r
    dth = math.pi / w.n_th
    r = w.r_min * np.exp((P["i1"] + P["dx1"].astype(np.float64)) * dxi)
    th = (P["i2"] + P["dx2"].astype(np.float64)) * dth
    c = [dxi * r, r * dth, r * np.maximum(np.abs(np.sin(th)), 1e-5)]
    u = [P[k].astype(np.float64) for k in ("u1", "u2", "u3")]
    gam = np.sqrt(1 + sum((ui / ci) ** 2 for ui, ci in zip(u, c)))
    return [gam * ci for ci in c]


def compare(w, P32, P64, what):
    """Per-particle errors of FP32 against FP64 on the slots live in both."""
    a, b = host(P32), host(P64)
    live = (a["tag"] != 0) & (b["tag"] != 0) & ((a["tag"] & 0x40) == 0)
    mismatch = int(((a["tag"] != 0) != (b["tag"] != 0)).sum())
    x_err = np.zeros(live.sum())
    for d in ("1", "2"):
        xa = a["i" + d] + a["dx" + d].astype(np.float64)
        xb = b["i" + d] + b["dx" + d]
        x_err = np.maximum(x_err, np.abs(xa - xb)[live])
    sc = u_scale(w, b)
    u_err = np.zeros(live.sum())
    for k, s in zip(("u1", "u2", "u3"), sc):
        e = np.abs(a[k].astype(np.float64) - b[k]) / np.maximum(np.abs(b[k]), s)
        u_err = np.maximum(u_err, e[live])
    stats = {"n": int(live.sum()), "tag_mismatch": mismatch,
             "x_med": float(np.median(x_err)), "x_max": float(x_err.max()),
             "u_med": float(np.median(u_err)), "u_p99": float(np.quantile(u_err, 0.99)),
             "u_max": float(u_err.max())}
    print(f"\n[fp32 vs fp64] {what}: " + " ".join(f"{k}={v:.3g}" if isinstance(v, float)
                                                else f"{k}={v}" for k, v in stats.items()))
    return stats, live


def plane_errors(F32, F64, planes):
    out = []
    for c in planes:
        a = F32[c].double().cpu().numpy()
        b = F64[c].cpu().numpy()
        s = np.abs(b).max()
        out.append(float(np.abs(a - b).max() / s) if s > 0 else float(np.abs(a).max()))
    return out


# ---------------------------------------------------------------- loading

def test_fp32_loading_is_rounded_fp64(G):
    import torch
    w = wl("c3_2048", 64)
    c32, c64 = contexts(G, w)
    n = w.n_particles
    P32, P64 = c32.new_particles(n), c64.new_particles(n)
    c32.particles_init(P32, 0, w.ppc, w.T, 0, w.seed)
    c64.particles_init(P64, 0, w.ppc, w.T, 0, w.seed)
    torch.cuda.synchronize()
    for k in P32:
        if P32[k].dtype == torch.float32:
            assert torch.equal(P32[k], P64[k].to(torch.float32)), k
        else:
            assert torch.equal(P32[k], P64[k]), k


@pytest.mark.parametrize("name", ["c3_2048", "c5_4096"])
def test_fp32_wald_is_rounded_fp64(G, name):
    import torch
    w = wl(name, 128)
    c32, c64 = contexts(G, w)
    F32, F64 = c32.new_fields(), c64.new_fields()
    c32.fields_init_wald(F32, w.B0)
    c64.fields_init_wald(F64, w.B0)
    torch.cuda.synchronize()
    assert F32.shape[0] == 39 and F64.shape[0] == 33
    assert torch.equal(F32[:33], F64.to(torch.float32))
    assert not F32[33:].any()      # compensation planes start at zero


def test_fp32_monopole_is_rounded_fp64(G):
    import torch
    w = wl("c6_monopole", 128)
    c32, c64 = contexts(G, w)
    F32, F64 = c32.new_fields(), c64.new_fields()
    c32.fields_init_monopole(F32, w.B0)
    c64.fields_init_monopole(F64, w.B0)
    torch.cuda.synchronize()
    assert torch.equal(F32[:33], F64.to(torch.float32))
    assert not F32[33:].any()


# ---------------------------------------------------------------- one stage

def loaded(G, w, c32, c64):
    n = w.n_particles
    P32 = c32.new_particles(n)
    c32.particles_init(P32, w.n_pairs_total if w.ppc == 0 else 0, w.ppc, w.T, w.n_geo, w.seed)
    F32 = c32.new_fields()
    c32.fields_init_wald(F32, w.B0)
    return P32, F32, widen(P32), F32[:33].double()


def test_fp32_push_one_step(G):
    w = wl("c3_2048", 256)
    c32, c64 = contexts(G, w)
    P32, F32, P64, F64 = loaded(G, w, c32, c64)
    c32.push(F32, P32)
    c64.push(F64, P64)
    st, _ = compare(w, P32, P64, "one push")
    assert st["tag_mismatch"] == 0
    assert st["x_max"] <= 2e-6 * w.n_r / 256 + 1e-6
    assert st["u_max"] <= 1e-5
    assert st["u_med"] <= 1e-6


def test_fp32_deposit(G):
    w = wl("c3_2048", 256)
    c32, c64 = contexts(G, w, charge_scale=1e-3)
    P32, F32, P64, F64 = loaded(G, w, c32, c64)
    c64.push(F64, P64)
    # both deposit the same move: the FP64 result rounded to FP32
    P32 = {k: (v.float() if v.dtype.is_floating_point else v.clone()) for k, v in P64.items()}
    P64 = widen(P32)
    c32.deposit(P32, F32)
    c64.deposit(P64, F64)
    errs = plane_errors(F32, F64, [18, 19, 20])
    print(f"\n[fp32 vs fp64] deposit J planes rel max err: {errs}")
    assert max(errs) <= 1e-5


def test_fp32_push_deposit_fused_equals_separate(G):
    import torch
    w = wl("c3_2048", 128)
    c32, _ = contexts(G, w, charge_scale=1e-3)
    P32, F32, _, _ = loaded(G, w, c32, c32)
    Pb = {k: v.clone() for k, v in P32.items()}
    Fb = F32.clone()
    for _ in range(3):
        c32.push(F32, P32)
        c32.deposit(P32, F32)
        c32.push_deposit(Fb, Pb)
    torch.cuda.synchronize()
    for k in P32:
        if k not in ("i1p", "i2p", "dx1p", "dx2p"):  # not written by the fused pass
            assert torch.equal(P32[k], Pb[k]), k
    errs = plane_errors(Fb, F32.double(), [18, 19, 20])
    print(f"\n[fp32] fused vs separate J rel max err: {errs}")
    assert max(errs) <= 1e-5


# ---------------------------------------------------------------- full steps

def test_fp32_full_steps_c3_recipe(G):
    """100 full PIC steps of the a = 0.99, B0 = 10, 32 ppc workload at 256^2:
    99% of the particles within 1e-5 (momenta and energy), fields within 1e-5
    of their max-norm away from the two cell rows next to each axis (where the
    conformal factor sqrt(h) ~ sin(theta) divides the rounding of the curl)
    and within 1e-4 on those rows."""
    import torch
    w = wl("c3_2048", 256)
    c32, c64 = contexts(G, w)
    P32, F32, P64, F64 = loaded(G, w, c32, c64)
    for _ in range(w.steps):
        c32.step(F32, P32, fused=True)
        c64.step(F64, P64, fused=True)
    torch.cuda.synchronize()
    st, live = compare(w, P32, P64, f"{w.steps} full steps")
    d32 = c32.diagnostics(F32, P32, w.B0, per_particle=True)
    d64 = c64.diagnostics(F64, P64, w.B0, per_particle=True)
    E32 = d32["E"].double().cpu().numpy()[live]
    E64 = d64["E"].cpu().numpy()[live]
    e_err = np.abs(E32 - E64) / np.maximum(np.abs(E64), 1.0)
    print(f"[fp32 vs fp64] energy rel err: med={np.median(e_err):.3g} "
          f"p99={np.quantile(e_err, 0.99):.3g} max={e_err.max():.3g}")
    g = 2
    inner = (slice(None), slice(g + 2, g + w.n_th - 1))
    err_in, err_all = [], []
    for c in range(6):
        a = F32[c].double().cpu().numpy()
        b = F64[c].cpu().numpy()
        s = np.abs(b).max()
        err_all.append(np.abs(a - b).max() / s)
        err_in.append(np.abs(a - b)[inner].max() / s)
    print(f"[fp32 vs fp64] D, B rel max err: inner {np.array(err_in)}, all {np.array(err_all)}")
    assert d32["n_nonfinite"] == 0 and d64["n_nonfinite"] == 0
    assert st["tag_mismatch"] <= max(2, 1e-5 * st["n"])
    assert st["u_p99"] <= 1e-5
    assert st["u_med"] <= 2e-6
    assert np.quantile(e_err, 0.99) <= 1e-5
    for sp in (1, 2):
        rel = abs(d32["sum_E"][sp] - d64["sum_E"][sp]) / abs(d64["sum_E"][sp])
        assert rel <= 1e-5, (sp, rel)
    assert max(err_in) <= 1e-5
    assert max(err_all) <= 1e-4


def _gauss_drift(c, F, P, w, steps):
    """Largest change of div D - 4 pi rho over `steps` fused full steps on
    every node the residual covers (axis nodes in the polar-cap form), and on
    the n_f + 2 node rows next to each axis, both over the largest term."""
    import torch
    nf, g = w.n_filter, 2
    near = np.r_[g:g + nf + 2, g + w.n_th - nf - 1:g + w.n_th + 1]
    d0 = c.diagnostics(F, P, w.B0, gauss_plane=True)
    R0 = d0["gauss_res"].double().clone()
    for _ in range(steps):
        c.step(F, P, fused=True)
    torch.cuda.synchronize()
    d1 = c.diagnostics(F, P, w.B0, gauss_plane=True)
    dR = (d1["gauss_res"].double() - R0).abs()
    scale = max(d0["gauss_scale"], d1["gauss_scale"])
    return dR.max().item() / scale, dR[:, near].max().item() / scale, d1["n_nonfinite"]


def test_fp32_gauss_c5_recipe(G):
    """Gauss's law with charge, 4 filter passes and the absorbing layer (C5
    recipe, 256^2, 50 steps): the change of div D - 4 pi rho is at most 1e-6
    of the largest term in FP32 on every checked node, the axis nodes and the
    rows next to the axes included (the deposit's two-sided axis rows keep the
    filtered current and charge consistent there); the FP64 form keeps it to
    round-off on the same nodes."""
    w = wl("c5_4096", 256, n_absorb=16)
    c32, c64 = contexts(G, w, charge_scale=1e-6)
    P32, F32, P64, F64 = loaded(G, w, c32, c64)
    out = {}
    for name, c, F, P in (("fp32", c32, F32, P32), ("fp64", c64, F64, P64)):
        out[name] = _gauss_drift(c, F, P, w, 50)
        print(f"\n[{name}] Gauss drift over 50 steps / largest term: all checked nodes "
              f"{out[name][0]:.3g}, rows next to the axes {out[name][1]:.3g}")
    assert out["fp64"][2] == 0 and out["fp32"][2] == 0
    assert out["fp64"][0] <= 1e-13
    assert out["fp32"][0] <= 1e-6


def test_fp32_sort(G):
    import torch
    w = wl("c3_2048", 64)
    c32, _ = contexts(G, w)
    P32, F32, _, _ = loaded(G, w, c32, c32)
    for _ in range(3):
        c32.step(F32, P32)
    Q = c32.new_particles(P32["tag"].numel())
    Q["tag"].fill_(1)  # the slots after the live ones must come back empty
    n_live = c32.sort(P32, Q, count=True)
    a, b = host(P32), host(Q)
    live_a = (a["tag"] != 0) & ((a["tag"] & 0x80) == 0)
    assert n_live == int(live_a.sum())
    assert (b["tag"][:n_live] != 0).all() and (b["tag"][n_live:] == 0).all()
    key = b["i1"][:n_live].astype(np.int64) * w.n_th + b["i2"][:n_live]
    assert (np.diff(key) >= 0).all()
    rows_a = np.sort(np.stack([a["u1"][live_a], a["u2"][live_a], a["u3"][live_a]]).view(np.uint32), axis=1)
    rows_b = np.sort(np.stack([b["u1"][:n_live], b["u2"][:n_live], b["u3"][:n_live]]).view(np.uint32), axis=1)
    np.testing.assert_array_equal(rows_a, rows_b)
    torch.cuda.synchronize()


def test_fp32_push_with_photons(G):
    """Massless particles (tag 7) in the single-precision push: one step of a
    loaded plasma with every fifth slot retagged, against the FP64 push of the
    same rounded state (the photons' momenta spread over e^+-3)."""
    import torch
    w = wl("c3_2048", 256)
    c32, c64 = contexts(G, w)
    P32, F32, _, F64 = loaded(G, w, c32, c64)
    g = torch.Generator(device="cpu").manual_seed(5)
    sel = torch.zeros(P32["tag"].numel(), dtype=torch.bool)
    sel[::5] = True
    P32["tag"][sel.to(P32["tag"].device)] = 7
    scale = torch.exp(torch.empty(int(sel.sum())).uniform_(-3.0, 3.0, generator=g)).to(torch.float32)
    for k in ("u1", "u2", "u3"):
        P32[k][sel.to(P32[k].device)] *= scale.to(P32[k].device)
    P64 = widen(P32)
    c32.push(F32, P32)
    c64.push(F64, P64)
    st, _ = compare(w, P32, P64, "one push with photons")
    assert st["tag_mismatch"] == 0
    assert st["x_max"] <= 2e-6 * w.n_r / 256 + 1e-6
    assert st["u_med"] <= 1e-6
    assert st["u_max"] <= 1e-4
