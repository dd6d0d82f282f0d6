"""Bounds guards of the push, forced from the host (every kernel exits
normally): slots with non-finite momenta or offsets, or a cell outside the
grid, end as tag 0x40 (dropped), are counted as non-finite by the
diagnostics, deposit nothing, and are left alone by later pushes; the sort
empties them.  Both precisions, fused and separate passes."""
import numpy as np
import pytest

from test_gpu_parity import G, pair, up, down, wl  # noqa: F401

pytestmark = pytest.mark.gpu

BAD = {  # slot -> (field, value) written on the host
    10: ("u1", np.nan), 11: ("u2", np.inf), 12: ("u3", -np.inf), 13: ("dx1", np.nan),
    14: ("i1", 40), 15: ("i2", -3), 16: ("dx2", 1.5), 17: ("i1", -2),
}


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("fused", [False, True])
def test_guards_drop_bad_slots(O, G, fp32, fused):
    import torch
    w = wl("c1_64", 32)
    prm, c64 = pair(O, G, w, charge_scale=0.1)
    ctx = G.Context(w.a, w.M, w.r_min, w.r_max, 32, 32, dt=c64.dt, charge_scale=0.1,
                    precision=G.GRPIC_FP32) if fp32 else c64
    F = O.fields_init_wald(prm, w.B0)
    P = O.particles_init(prm, 200, 0, 1.0, 0, 5)
    Pbad = {k: v.copy() for k, v in P.items()}
    for q, (f, v) in BAD.items():
        Pbad[f][q] = v
    Pref = {k: v.copy() for k, v in P.items()}
    Pref["tag"][list(BAD)] = 0                  # the same set with those slots empty

    def run(Ph):
        Pg = up(Ph)
        Fg = up({"F": F})["F"]
        if fp32:
            Pg = {k: (v.float() if v.is_floating_point() else v) for k, v in Pg.items()}
            F32 = ctx.new_fields()
            F32[:33] = Fg.float()
            Fg = F32
        if fused:
            ctx.push_deposit(Fg, Pg)
        else:
            ctx.push(Fg, Pg)
            ctx.deposit(Pg, Fg)
        torch.cuda.synchronize()
        return Pg, Fg

    Pg, Fg = run(Pbad)
    Pr, Fr = run(Pref)
    tags = Pg["tag"].cpu().numpy()
    assert (tags[list(BAD)] == 0x40).all()
    good = np.setdiff1d(np.arange(len(tags)), list(BAD))
    for k in ("tag", "i1", "i2", "dx1", "dx2", "u1", "u2", "u3"):
        np.testing.assert_array_equal(Pg[k].cpu().numpy()[good], Pr[k].cpu().numpy()[good], err_msg=k)
    for c in (18, 19, 20):  # the dropped slots deposited nothing (atomics: summation order varies)
        a, b = Fg[c].double().cpu().numpy(), Fr[c].double().cpu().numpy()
        tol = (1e-6 if fp32 else 1e-14) * np.abs(b).max()
        assert np.abs(a - b).max() <= tol, c
    d = ctx.diagnostics(Fg, Pg, w.B0)
    assert d["n_nonfinite"] == len(BAD)
    before = {k: v.clone() for k, v in Pg.items()}
    ctx.push(Fg, Pg)                            # dropped slots stay as they are
    torch.cuda.synchronize()
    for k in ("tag", "i1", "i2", "dx1", "dx2", "u1", "u2", "u3"):
        a, b = Pg[k].cpu().numpy()[list(BAD)], before[k].cpu().numpy()[list(BAD)]
        np.testing.assert_array_equal(a, b, err_msg=k)
    Q = ctx.new_particles(len(tags))
    n_live = ctx.sort(Pg, Q, count=True)
    qt = Q["tag"].cpu().numpy()
    assert (qt[:n_live] != 0).all() and (qt[:n_live] & 0x40 == 0).all() and (qt[n_live:] == 0).all()
