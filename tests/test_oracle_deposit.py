"""Pins of the oracle's conformal charge-conserving deposit (Sec. 3.2)."""
import math

import numpy as np
import pytest

from _helpers import grid


def params(O, n=16, dt=0.1, kappa=1.0):
    return O.Params.make(0.9, 1.0, 1.3, 20.0, n, n, dt, charge_scale=kappa)


def moved_particles(O, prm, n, seed):
    """Random previous positions and moves of up to 0.75 cell per dimension."""
    g = np.random.default_rng(seed)
    P = O.new_particles(n)
    P["i1p"][:] = g.integers(2, prm.n_r - 2, n)
    P["i2p"][:] = g.integers(2, prm.n_th - 2, n)
    P["dx1p"][:] = g.random(n)
    P["dx2p"][:] = g.random(n)
    x1 = P["i1p"] + P["dx1p"] + g.uniform(-0.75, 0.75, n)
    x2 = P["i2p"] + P["dx2p"] + g.uniform(-0.75, 0.75, n)
    P["i1"][:] = np.floor(x1); P["dx1"][:] = x1 - np.floor(x1)
    P["i2"][:] = np.floor(x2); P["dx2"][:] = x2 - np.floor(x2)
    P["u1"][:] = g.normal(size=n) * 0.01
    P["u2"][:] = g.normal(size=n) * 0.01
    P["u3"][:] = g.normal(size=n)
    P["w"][:] = g.uniform(0.5, 2.0, n)
    P["tag"][:] = g.integers(1, 3, n)
    return P


def charge_at(O, prm, P, prev):
    Q = {k: v.copy() for k, v in P.items()}
    if prev:
        for c in ("i1", "i2", "dx1", "dx2"):
            Q[c] = P[c + "p"].copy()
    return O.charge(prm, Q)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_continuity_per_particle(O, seed):
    """Discrete continuity (eq. charge-conservation-disc): for every particle
    and at every node, [S(x^{n+1}) - S(x^n)] q + dt div(J) = 0 to round-off,
    including moves across cell edges in both directions and corners."""
    prm = params(O)
    Pall = moved_particles(O, prm, 200, seed)
    for k in range(200):
        P = {c: v[k:k + 1].copy() for c, v in Pall.items()}
        F = O.new_fields(prm)
        O.deposit(prm, F, P)
        J1, J2 = F[O.PLANES["J"]], F[O.PLANES["J"] + 1]
        div = J1.copy()
        div[1:, :] -= J1[:-1, :]
        div[:, 1:] += J2[:, 1:] - J2[:, :-1]
        div[:, 0] += J2[:, 0]
        drho = charge_at(O, prm, P, False) - charge_at(O, prm, P, True)
        res = drho + prm.dt * div
        assert np.abs(res).max() <= 1e-14 * max(1.0, np.abs(drho).max()), k


def test_zigzag_hand_values(O):
    """Umeda et al. (2003) zigzag for a move inside one cell, q = 1, dt = 1,
    from (0.2, 0.3) to (0.6, 0.5) in cell (5, 7): relay at the midpoint,
    J1(5+1/2, 7) = 0.2*0.65 + 0.2*0.55 = 0.24, J1(5+1/2, 8) = 0.16,
    J2(5, 7+1/2) = 0.1*0.7 + 0.1*0.5 = 0.12, J2(6, 7+1/2) = 0.08."""
    prm = params(O, dt=1.0)
    P = O.new_particles(1)
    P["i1p"][0], P["i2p"][0], P["dx1p"][0], P["dx2p"][0] = 5, 7, 0.2, 0.3
    P["i1"][0], P["i2"][0], P["dx1"][0], P["dx2"][0] = 5, 7, 0.6, 0.5
    P["w"][0], P["tag"][0] = 1.0, 1
    F = O.new_fields(prm)
    O.deposit(prm, F, P)
    g = prm.ng
    J1, J2 = F[O.PLANES["J"]], F[O.PLANES["J"] + 1]
    assert J1[5 + g, 7 + g] == pytest.approx(0.24, abs=1e-15)
    assert J1[5 + g, 8 + g] == pytest.approx(0.16, abs=1e-15)
    assert J2[5 + g, 7 + g] == pytest.approx(0.12, abs=1e-15)
    assert J2[6 + g, 7 + g] == pytest.approx(0.08, abs=1e-15)
    assert np.count_nonzero(J1) == 2 and np.count_nonzero(J2) == 2
    # crossing one edge in x1: relay point on the edge
    P["i1"][0], P["dx1"][0], P["dx2"][0] = 6, 0.1, 0.3
    F = O.new_fields(prm)
    O.deposit(prm, F, P)
    J1 = F[O.PLANES["J"]]
    # segment 1: 0.2 -> 1.0 at y = 0.3 in cell 5; segment 2: 0 -> 0.1 in cell 6
    assert J1[5 + g, 7 + g] == pytest.approx(0.8 * 0.7, abs=1e-15)
    assert J1[6 + g, 7 + g] == pytest.approx(0.1 * 0.7, abs=1e-15)


def test_out_of_plane_current(O):
    """J^3 = q alpha u^3 / gamma at the path midpoint with first-order shape
    weights that sum to one (Sec. 3.2); theta clamped near the axis (Sec. 3.3.2)."""
    prm = params(O, kappa=0.5)
    P = moved_particles(O, prm, 1, 11)
    P["tag"][0], P["w"][0] = 2, 1.5
    F = O.new_fields(prm)
    O.deposit(prm, F, P)
    x1 = 0.5 * (P["i1p"][0] + P["dx1p"][0] + P["i1"][0] + P["dx1"][0])
    x2 = 0.5 * (P["i2p"][0] + P["dx2p"][0] + P["i2"][0] + P["dx2"][0])
    m = O.metric_at(prm, x1, x2)
    u = [P["u1"][0], P["u2"][0], P["u3"][0]]
    gam = math.sqrt(1 + m["hu11"] * u[0] ** 2 + m["hu22"] * u[1] ** 2 + m["hu33"] * u[2] ** 2 +
                    2 * m["hu13"] * u[0] * u[2])
    vphi = m["alpha"] * (m["hu13"] * u[0] + m["hu33"] * u[2]) / gam
    J3 = F[O.PLANES["J"] + 2]
    assert J3.sum() == pytest.approx(-0.5 * 1.5 * vphi, rel=1e-13)
    assert np.count_nonzero(J3) == 4


def test_neutral_and_dead_deposit_nothing(O):
    prm = params(O)
    P = moved_particles(O, prm, 50, 5)
    P["tag"][:25] = 3
    P["tag"][25:] = 0
    F = O.new_fields(prm)
    O.deposit(prm, F, P)
    assert not F.any()


def test_linear_in_weight_and_order_independent(O):
    """Deposit sums over particles: doubling weights doubles J; reversing the
    particle order changes J by round-off only."""
    prm = params(O)
    P = moved_particles(O, prm, 300, 3)
    F1 = O.new_fields(prm)
    O.deposit(prm, F1, P)
    R = {k: v[::-1].copy() for k, v in P.items()}
    F2 = O.new_fields(prm)
    O.deposit(prm, F2, R)
    sl = slice(O.PLANES["J"], O.PLANES["J"] + 3)
    np.testing.assert_allclose(F1[sl], F2[sl], rtol=0, atol=1e-13 * np.abs(F1[sl]).max())
    P["w"] *= 2
    F3 = O.new_fields(prm)
    O.deposit(prm, F3, P)
    np.testing.assert_allclose(F3[sl], 2 * F1[sl], rtol=0, atol=1e-13 * np.abs(F1[sl]).max())
