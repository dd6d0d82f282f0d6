"""Pair injection on the GPU (grpic_inject_pairs, Sec. 4.4 and Sec. 4.5)
against the oracle, through the C ABI.

Both sides start from one oracle-made state (Wald field, loaded plasma with
some slots emptied); the threshold is a quantile of the oracle's sigma, moved
off any cell whose sigma lies within 1e-9 of it (the decision is taken in FP64
on both sides, from sums in different orders).  Compared: the count, tags,
cells and offsets bit for bit, momenta to 1e-12 of the particle's scale (FP64
form); in the FP32 form the oracle runs on the state widened from FP32 and the
results are compared after rounding to float (offsets exact, momenta to
2 ulp).  Also: two calls in a row (the second from where the first ended),
capacity (whole pairs only) and Gauss's law unchanged by the injection.
"""
import numpy as np
import pytest

from test_gpu_parity import G, pair, up, down, u_scale, wl  # noqa: F401

pytestmark = pytest.mark.gpu


def state(O, prm, n_pairs, room, seed=3):
    P0 = O.particles_init(prm, n_pairs, 0, 1.0, 0, seed)
    P0["tag"][1::2][::3] = 0                   # emptied slots: net charge, uneven density
    P0["tag"][::17] |= 0x80                    # leaving slots do not count
    n0 = len(P0["tag"])
    P = O.new_particles(n0 + room)
    for k in P0:
        P[k][:n0] = P0[k]
    return P, n0


def threshold(O, prm, F, P, q):
    sig = O.magnetisation(prm, F, P)
    fin = sig[np.isfinite(sig) & (sig > 0)]
    th = float(np.quantile(fin, q))
    while (np.abs(fin / th - 1) < 1e-9).any():
        th *= 1 + 1e-7
    return th


def widen(P):
    return {k: (v.astype(np.float64) if v.dtype == np.float32 else v.copy()) for k, v in P.items()}


def narrow(P):
    return {k: (v.astype(np.float32) if v.dtype == np.float64 else v.copy()) for k, v in P.items()}


def compare(prm, Po, Pg, n0, k, f32=False):
    sl = slice(n0, n0 + 2 * k)
    for c in ("tag", "i1", "i2", "i1p", "i2p"):
        np.testing.assert_array_equal(Pg[c][sl], Po[c][sl], err_msg=c)
    assert (Pg["tag"][n0 + 2 * k:] == 0).all()
    for c in ("dx1", "dx2", "dx1p", "dx2p", "w", "phi"):
        ref = Po[c][sl].astype(np.float32) if f32 else Po[c][sl]
        np.testing.assert_array_equal(Pg[c][sl], ref, err_msg=c)
    sc = u_scale(prm, {c: Po[c][sl] for c in ("i1", "i2", "dx1", "dx2", "u1", "u2", "u3")})
    for c, s in zip(("u1", "u2", "u3"), sc):
        err = np.abs(Pg[c][sl].astype(np.float64) - Po[c][sl]) / s
        bar = 2 * 2.0 ** -23 if f32 else 1e-12
        assert err.max(initial=0) <= bar, f"{c} err {err.max():.3g}"


@pytest.mark.parametrize("n_inj", [1, 4])
def test_inject_parity_fp64(O, G, n_inj):
    """C1 recipe at 48^2, a = 0.9: one injection call against the oracle."""
    w = wl("c1_64", 48)
    prm, ctx = pair(O, G, w, charge_scale=1e-3)
    F = O.fields_init_wald(prm, w.B0)
    P, n0 = state(O, prm, 3000, 2 * n_inj * 48 * 48)
    th = threshold(O, prm, F, P, 0.4)
    Pg = up(P)
    Fg = up({"F": F})["F"]
    k = O.inject_pairs(prm, F, P, th, 0.5, n_inj, 0.75, 2, 44, 21, 0, n0)
    kg = ctx.inject_pairs(Fg, Pg, th, 0.5, n_inj, 0.75, 2, 44, 21, 0, n0)
    print(f"\n[inject fp64] {k} pairs (oracle), {kg} (GPU), threshold {th:.4g}")
    assert k > 100 and kg == k
    Pd = down(Pg)
    compare(prm, P, Pd, n0, k)
    for c in P:                                 # the slots before first_free are untouched
        np.testing.assert_array_equal(Pd[c][:n0], P[c][:n0], err_msg=c)


def test_inject_two_calls_and_capacity(O, G):
    """Two calls in a row (call 0, then call 1 from the first free slot after
    the first), the second running out of room mid-way: counts, slots and
    values as the oracle's."""
    w = wl("c1_64", 32)
    prm, ctx = pair(O, G, w, charge_scale=1e-3)
    F = O.fields_init_wald(prm, w.B0)
    P, n0 = state(O, prm, 1000, 1500)
    th = threshold(O, prm, F, P, 0.5)
    Pg, Fg = up(P), up({"F": F})["F"]
    k1 = O.inject_pairs(prm, F, P, th, 0.5, 1, 1.0, 0, 32, 5, 0, n0)
    g1 = ctx.inject_pairs(Fg, Pg, th, 0.5, 1, 1.0, 0, 32, 5, 0, n0)
    assert g1 == k1 and 2 * k1 < 1500
    f2 = n0 + 2 * k1
    k2 = O.inject_pairs(prm, F, P, th, 0.5, 2, 1.0, 0, 32, 5, 1, f2)
    g2 = ctx.inject_pairs(Fg, Pg, th, 0.5, 2, 1.0, 0, 32, 5, 1, f2)
    room = len(P["tag"]) - f2
    print(f"\n[inject twice] {k1} then {k2} pairs (room for {room // 2})")
    assert g2 == k2 == room // 2
    compare(prm, P, down(Pg), n0, k1 + k2)


def test_inject_parity_fp32(O, G):
    """FP32 form (C5 recipe at 64^2, absorbing layer 8): the oracle injects
    into the state widened from the GPU's FP32 copy of the same input."""
    import torch
    w = wl("c5_4096", 64, n_absorb=8)
    prm, c64 = pair(O, G, w, charge_scale=1e-3)
    c32 = G.Context(w.a, w.M, w.r_min, w.r_max, 64, 64, dt=c64.dt, n_iter=w.n_iter,
                    small_angle=w.small_angle, charge_scale=1e-3, n_filter=w.n_filter,
                    n_absorb=8, precision=G.GRPIC_FP32)
    F = O.fields_init_wald(prm, w.B0)
    P, n0 = state(O, prm, 4000, 6000)
    F32 = c32.new_fields()
    F32[:33] = torch.from_numpy(F).to(torch.float32).cuda()
    P32 = up(narrow(P))
    Fw = F32[:33].double().cpu().numpy().copy()
    Pw = widen(down(P32))
    th = threshold(O, prm, Fw, Pw, 0.4)
    k = O.inject_pairs(prm, Fw, Pw, th, 0.5, 2, 1.0, 0, 64, 8, 2, n0)
    kg = c32.inject_pairs(F32, P32, th, 0.5, 2, 1.0, 0, 64, 8, 2, n0)
    print(f"\n[inject fp32] {k} pairs (oracle on the widened state), {kg} (GPU)")
    assert k > 100 and kg == k
    compare(prm, Pw, down(P32), n0, k, f32=True)


def test_inject_keeps_gauss(O, G):
    """Co-located pairs carry no net charge: the GPU's Gauss residual (with
    n_f = 2) is the same before and after an injection, to round-off of the
    largest term."""
    w = wl("c1_64", 32)
    prm, ctx = pair(O, G, w, charge_scale=1e-3, n_filter=2)
    F = O.fields_init_wald(prm, w.B0)
    P, n0 = state(O, prm, 1000, 3000)
    Pg, Fg = up(P), up({"F": F})["F"]
    d0 = ctx.diagnostics(Fg, Pg, w.B0, gauss_plane=True)
    R0 = d0["gauss_res"].clone()
    # sigma = 1e300: only the empty magnetised cells (sigma = infinity) inject
    k1 = ctx.inject_pairs(Fg, Pg, 1e300, 0.5, 1, 1.0, 0, 32, 1, 0, n0)
    assert k1 == int(np.isinf(O.magnetisation(prm, F, P)).sum()) > 0
    k2 = ctx.inject_pairs(Fg, Pg, threshold(O, prm, F, P, 0.5), 0.5, 1, 1.0, 0, 32, 1, 1,
                          n0 + 2 * k1)
    assert k2 > 50
    k = k1 + k2
    d1 = ctx.diagnostics(Fg, Pg, w.B0, gauss_plane=True)
    assert d1["n_alive"][1] - d0["n_alive"][1] == k and d1["n_alive"][2] - d0["n_alive"][2] == k
    dR = (d1["gauss_res"] - R0).abs().max().item()
    assert dR <= 1e-13 * max(d0["gauss_scale"], d1["gauss_scale"])


def test_inject_rejects_bad_arguments(O, G):
    """Host-side argument checks: first_free outside the set, a non-positive
    threshold or temperature, negative pair counts."""
    w = wl("c1_64", 16)
    prm, ctx = pair(O, G, w)
    Fg = ctx.new_fields()
    Pg = ctx.new_particles(10)
    for kw in ({"first_free": 11}, {"first_free": -1}, {"sigma_th": 0.0},
               {"temperature": -1.0}, {"n_pairs": -1}):
        args = dict(sigma_th=1.0, temperature=0.5, n_pairs=1, weight=1.0, i_lo=0, i_hi=16,
                    seed=0, call=0, first_free=0)
        args.update(kw)
        with pytest.raises(G.GrpicError):
            ctx.inject_pairs(Fg, Pg, **args)
