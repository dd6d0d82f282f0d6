"""Pins of the oracle's particle update (Sec. 3.1) against closed forms,
conservation laws and special cases (no GPU)."""
import math

import numpy as np
import pytest

from _helpers import cartesian, fit_circle, grid, place, position, single


def params(O, a, M, r_min, r_max, n, dt, n_iter=10):
    return O.Params.make(a, M, r_min, r_max, n, n, dt, n_iter=n_iter)


# -------------------------------------------------------------------- Boris

def test_boris_magnetic_rotation_closed_form(O):
    """Pure magnetic Boris step: |u| is preserved and u rotates about B by the
    angle 2 atan(qm tau |B| / (2 gamma)) (Boris 1970)."""
    g = np.random.default_rng(5)
    for _ in range(50):
        u = g.normal(size=3) * 3
        B = g.normal(size=3)
        qm = g.choice([-1.0, 1.0])
        tau = g.uniform(0.01, 0.5)
        un = O.boris(u, [0, 0, 0], B, qm, tau)
        gam = math.sqrt(1 + u @ u)
        Bn = np.linalg.norm(B)
        ang = 2 * math.atan(qm * tau * Bn / (2 * gam))
        n = B / Bn
        # rotation of u by -ang about n (du/dt = qm u x B / gamma)
        ref = (u * math.cos(ang) + np.cross(u, n) * math.sin(ang) +
               n * (n @ u) * (1 - math.cos(ang)))
        np.testing.assert_allclose(un, ref, rtol=1e-13, atol=1e-13 * np.abs(u).max())


def test_boris_electric_only(O):
    """With B = 0 the Boris step is u + qm tau E exactly."""
    u = np.array([0.3, -1.2, 2.0])
    E = np.array([0.5, 0.25, -1.0])
    un = O.boris(u, E, [0, 0, 0], -1.0, 0.125)
    np.testing.assert_allclose(un, u - 0.125 * E, rtol=0, atol=1e-15)


# -------------------------------------------------------- flat-space orbits

def test_flat_gyration_circle(O):
    """SR-EM row of Table 1 (flat metric, vertical field B0 = 0.5, u_phi = 10 at
    r = 10): a circle of radius u_phihat/(qm B0) = 2 in the equatorial plane with
    period 2 pi gamma/(qm B0) = 4 pi sqrt 2 (Sec. 4.1.2)."""
    prm = params(O, 0.0, 0.0, 0.9, 20.0, 256, 0.01)
    dxi, dth = grid(0.9, 20.0, 256, 256)
    F = O.fields_init_wald(prm, 0.5)
    P = single(O, prm, 10.0, math.pi / 2, 0.0, 0.0, 10.0, 1)
    xs = []
    steps = int(round(4 * math.pi * math.sqrt(2) / 0.01))
    for _ in range(steps):
        O.push(prm, F, P)
        r, th = position(P, 0, 0.9, dxi, dth)
        xs.append(cartesian(r, th, P["phi"][0]))
    xs = np.array(xs)
    cx, cy, rad = fit_circle(xs[:, 0], xs[:, 1])
    assert rad == pytest.approx(2.0, rel=2e-3)
    assert abs(xs[:, 2]).max() < 1e-12
    rr = np.hypot(xs[:, 0] - cx, xs[:, 1] - cy)
    assert rr.max() - rr.min() < 5e-3
    # after one period the particle is back where it started (phase error O(dt^2))
    x0 = cartesian(10.0, math.pi / 2, 0.0)
    assert np.linalg.norm(xs[-1] - x0) < 0.02
    E, _ = O.energy_momentum(prm, P, 0.5)
    assert E[0] == pytest.approx(math.sqrt(2.0), rel=1e-6)


def test_flat_free_motion_is_straight(O):
    """A free particle in flat space (M = 0) moves on a straight line at
    constant velocity in Cartesian coordinates; the curvilinear geodesic
    momentum and coordinate iterations must reproduce it to O(dt^2).  The
    leapfrog needs u at t = -dt/2 (Sec. 3.1 staggering): its covariant spherical
    components are taken at the trajectory point x(-dt/2)."""
    errs = []
    for dt in (0.02, 0.01):
        prm = params(O, 0.0, 0.0, 0.5, 40.0, 256, dt)
        dxi, dth = grid(0.5, 40.0, 256, 256)
        x0 = cartesian(12.0, 1.0, 0.0)
        v = np.array([0.25, 0.45, -0.3])
        gam = 1.0 / math.sqrt(1.0 - v @ v)
        xh = x0 - 0.5 * dt * v
        rh = np.linalg.norm(xh)
        thh = math.acos(xh[2] / rh)
        phh = math.atan2(xh[1], xh[0])
        st, ct, sp_, cp = math.sin(thh), math.cos(thh), math.sin(phh), math.cos(phh)
        er = np.array([st * cp, st * sp_, ct])
        et = np.array([ct * cp, ct * sp_, -st])
        ep = np.array([-sp_, cp, 0.0])
        P = single(O, prm, 12.0, 1.0, 0.0, 0.0, 0.0, 3)
        P["u1"][0] = gam * (v @ er) * dxi * rh
        P["u2"][0] = gam * (v @ et) * rh * dth
        P["u3"][0] = gam * (v @ ep) * rh * st
        n = int(round(10.0 / dt))
        F = np.zeros((33,) + prm.shape())
        for _ in range(n):
            O.push(prm, F, P)
        r, th = position(P, 0, 0.5, dxi, dth)
        xe = cartesian(r, th, P["phi"][0])
        errs.append(np.linalg.norm(xe - (x0 + v * n * dt)))
    assert errs[1] < 2e-5
    assert 3.0 < errs[0] / errs[1] < 5.0


# ------------------------------------------------------------ GR geodesics

def test_neutral_u3_exact_and_energy_second_order(O):
    """Neutral particles: u_3 is bit-for-bit unchanged (eq. discretized-geodesic-u)
    and the energy error of the Table 1 GR orbit is bounded and second order
    in dt (halving dt cuts it by about 4)."""
    from _helpers import bl_energy
    a = 0.995
    E0, u_r = bl_energy(a, 1.0, 10.6498, math.pi / 2, 2.0)
    rh = 1 + math.sqrt(1 - a * a)
    errs = []
    for dt in (0.04, 0.02):
        prm = params(O, a, 1.0, 0.9 * rh, 15.0, 512, dt)
        P = single(O, prm, 10.6498, math.pi / 2, u_r, 0.0, 2.0, 3)
        F = np.zeros((33,) + prm.shape())
        e = 0.0
        for _ in range(int(round(60.0 / dt))):
            O.push(prm, F, P)
            assert P["u3"][0] == 2.0
            E, _ = O.energy_momentum(prm, P, 0.0)
            e = max(e, abs(E[0] / E0 - 1))
        errs.append(e)
    assert errs[1] < 1e-6
    assert 3.3 < errs[0] / errs[1] < 4.7


def test_iterations_converge(O):
    """The fixed-point iterations of eq. discretized-geodesic-u/-x converge to the
    implicit-midpoint solution: 30 and 40 iterations agree to round-off, and the
    paper's default of ten is within 1e-8 of the limit on the coarse 64^2 grid away
    from the axis, and within 1e-4 next to it
    (slowest contraction, about 0.3 per iteration, within a few 1e-4 rad of the
    axis where h^33 ~ 1/sin^2)."""
    a = 0.9
    rh = 1 + math.sqrt(1 - a * a)
    out = {}
    for n_iter in (10, 30, 40):
        prm = params(O, a, 1.0, 0.9 * rh, 20.0, 64, 0.0215869, n_iter=n_iter)
        F = O.fields_init_wald(prm, 1.0)
        P = O.particles_init(prm, 400, 0, 1.0, 0, 7)
        O.push(prm, F, P)
        out[n_iter] = P
    for k in ("u1", "u2", "u3", "dx1", "dx2"):
        sc = np.abs(out[40][k]).max()
        np.testing.assert_allclose(out[30][k], out[40][k], rtol=1e-13, atol=1e-14 * sc)
        np.testing.assert_allclose(out[10][k], out[40][k], rtol=1e-4, atol=1e-5 * sc)
        off_axis = (out[40]["i2p"] > 2) & (out[40]["i2p"] < 61)
        np.testing.assert_allclose(out[10][k][off_axis], out[40][k][off_axis], rtol=1e-8,
                                   atol=1e-9 * sc)
    np.testing.assert_array_equal(out[30]["i1"], out[40]["i1"])


def test_charged_wald_orbit_conserves_E_L(O):
    """GR-EM-2D row (a = 0, Wald/vertical field, calB = 0.1): E and L of the
    charged particle stay constant up to the interpolation drift (Sec. 4.1.3)."""
    from _helpers import bl_energy
    E0, u_r = bl_energy(0.0, 1.0, 4.0, math.pi / 2, 2.9)
    prm = params(O, 0.0, 1.0, 1.8, 20.0, 512, 0.01)
    F = O.fields_init_wald(prm, 0.2)
    P = single(O, prm, 4.0, math.pi / 2, u_r, 0.0, 2.9, 1)
    Es, Ls = [], []
    for _ in range(3000):
        O.push(prm, F, P)
        E, L = O.energy_momentum(prm, P, 0.2)
        Es.append(E[0]); Ls.append(L[0])
    assert max(abs(np.array(Es) / E0 - 1)) < 2e-4
    assert max(abs(np.array(Ls) / 4.5 - 1)) < 2e-4


# -------------------------------------------------------- boundaries, edge

def test_axis_reflection(O):
    """A particle crossing theta = 0 (or pi) is reflected: i2 reset to 0 (or
    N_theta - 1), dx2 -> 1 - dx2, u_2 -> -u_2 (Sec. 3.3.3).  In flat space the
    two axes mirror each other."""
    prm = params(O, 0.0, 0.0, 1.0, 20.0, 64, 0.05)
    dxi, dth = grid(1.0, 20.0, 64, 64)
    F = np.zeros((33,) + prm.shape())
    P = single(O, prm, 5.0, 0.05 * dth, 0.0, -0.8 * 5.0, 0.0, 3)
    u2_0 = P["u2"][0]
    O.push(prm, F, P)
    assert P["i2"][0] == 0 and 0.0 < P["dx2"][0] < 0.5
    assert P["u2"][0] > 0 and P["u2"][0] == pytest.approx(-u2_0, rel=1e-3)
    Q = single(O, prm, 5.0, math.pi - 0.05 * dth, 0.0, 0.8 * 5.0, 0.0, 3)
    O.push(prm, F, Q)
    assert Q["i2"][0] == 63
    assert Q["dx2"][0] == pytest.approx(1.0 - P["dx2"][0], abs=1e-9)
    assert Q["u2"][0] == pytest.approx(-P["u2"][0], rel=1e-9)
    assert Q["i1"][0] == P["i1"][0] and Q["dx1"][0] == pytest.approx(P["dx1"][0], abs=1e-12)


def test_removal_after_deposit(O):
    """A particle entering the inner ghost zone (i1 < 0) keeps its slot for the
    deposit of that step (leaving flag) and is removed by the next push."""
    prm = params(O, 0.9, 1.0, 0.9 * (1 + math.sqrt(1 - 0.81)), 20.0, 64, 0.02)
    dxi, dth = grid(prm.r_min, 20.0, 64, 64)
    P = single(O, prm, prm.r_min * math.exp(0.1 * dxi), 1.2, -3.0, 0.0, 0.0, 2)
    F = np.zeros((33,) + prm.shape())
    O.push(prm, F, P)
    assert P["i1"][0] < 0 and P["tag"][0] == (2 | O.TAG_LEAVING)
    O.push(prm, F, P)
    assert P["tag"][0] == 0


def test_dead_particles_untouched(O):
    prm = params(O, 0.9, 1.0, 1.2, 20.0, 64, 0.02)
    P = O.particles_init(prm, 10, 0, 1.0, 0, 3)
    P["tag"][:] = 0
    ref = {k: v.copy() for k, v in P.items()}
    O.push(prm, O.fields_init_wald(prm, 1.0), P)
    for k in P:
        np.testing.assert_array_equal(P[k], ref[k])


# ---------------------------------------------------------- massless (Sec. 2.3)

def _photon_orbit(a, M, prograde):
    """Equatorial circular photon orbit of Kerr: radius and impact parameter
    b = L/E (Bardeen, Press & Teukolsky 1972), the angular velocity
    dphi/dt = u^phi / u^t from the Boyer-Lindquist inverse metric, and the
    Kerr-Schild u_r of eq. BL-KS-transformation for E = 1."""
    s = -1.0 if prograde else 1.0
    c = math.cos(math.acos(s * a / M) / 3.0)
    r = 2.0 * M * (1.0 + math.cos(2.0 / 3.0 * math.acos(s * a / M)))
    b = -a - s * 6.0 * M * c
    Sig, Del = r * r, r * r - 2 * M * r + a * a
    gtt, gtp = -(1 - 2 * M * r / Sig), -2 * M * a * r / Sig
    gpp = r * r + a * a + 2 * M * a * a * r / Sig
    det = gtt * gpp - gtp * gtp
    Gtt, Gtp, Gpp = gpp / det, -gtp / det, gtt / det
    assert abs(Gtt - 2 * Gtp * b + Gpp * b * b) < 1e-12   # null at u_r(BL) = 0
    om = (-Gtp + Gpp * b) / (-Gtt + Gtp * b)
    return r, b, om, -(-2 * M * r + a * b) / Del


@pytest.mark.parametrize("a,prograde", [(0.0, True), (0.9, True), (0.9, False)])
def test_photon_circular_orbit(O, a, prograde):
    """Massless particles (tag species 3 + bit 0x04, gamma = sqrt(h^ij u_i u_j)):
    the equatorial circular photon orbit is a fixed point of both implicit
    updates, so the radius holds to round-off and phi advances at the orbit's
    angular velocity; the same momentum on a massive neutral particle (the
    mass term kept) leaves the orbit at once."""
    M = 1.0
    r, b, om, u_r = _photon_orbit(a, M, prograde)
    rh = 1 + math.sqrt(1 - a * a)
    r_min = 0.9 * rh
    dxi, dth = grid(r_min, 12.0, 512, 512)
    prm = params(O, a, M, r_min, 12.0, 512, 0.01)
    F = np.zeros((33,) + prm.shape())
    P = single(O, prm, r, math.pi / 2, u_r, 0.0, b, 7)
    Q = single(O, prm, r, math.pi / 2, u_r, 0.0, b, 3)
    dr = dq = 0.0
    n = 2000
    for _ in range(n):
        O.push(prm, F, P)
        O.push(prm, F, Q)
        dr = max(dr, abs(position(P, 0, r_min, dxi, dth)[0] / r - 1))
        if Q["tag"][0]:
            dq = max(dq, abs(position(Q, 0, r_min, dxi, dth)[0] / r - 1))
    assert P["tag"][0] == 7
    assert dr < 1e-13
    assert abs(P["phi"][0] - om * n * prm.dt) < 1e-11 * n * prm.dt
    assert dq > 1e-2


def test_photon_energy_second_order_and_L_exact(O):
    """A photon scattered by a Kerr hole (a = 0.9, closest approach r ~ 4):
    u_3 = L stays bit-for-bit, and the conserved E at the time-centred
    positions drifts at second order in dt."""
    a = 0.9
    rh = 1 + math.sqrt(1 - a * a)
    errs = []
    for dt in (0.04, 0.02):
        prm = params(O, a, 1.0, 0.9 * rh, 40.0, 512, dt)
        P = single(O, prm, 12.0, 1.2, -1.0, 0.6, 5.0, 7)
        F = np.zeros((33,) + prm.shape())
        O.push(prm, F, P)
        E0, _ = O.energy_momentum(prm, P, 0.0)
        e = 0.0
        for _ in range(int(round(40.0 / dt))):
            O.push(prm, F, P)
            E, L = O.energy_momentum(prm, P, 0.0)
            assert L[0] == 5.0
            e = max(e, abs(E[0] / E0[0] - 1))
        assert P["tag"][0] == 7
        errs.append(e)
    assert errs[1] < 1e-6
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_photon_scale_invariance_bit_exact(O):
    """Null geodesics do not depend on the scale of the momentum: doubling u
    (a power of two, so every rounding scales with it) gives the same path to
    the last bit and exactly twice the momentum; a massive particle does not
    share the property."""
    a = 0.9
    rh = 1 + math.sqrt(1 - a * a)
    prm = params(O, a, 1.0, 0.9 * rh, 40.0, 256, 0.02)
    F = np.zeros((33,) + prm.shape())
    for tag, same in ((7, True), (3, False)):
        Ps = [single(O, prm, 8.0, 1.0, -0.7 * s, 0.4 * s, 3.0 * s, tag) for s in (1, 2)]
        for _ in range(300):
            for P in Ps:
                O.push(prm, F, P)
        pos = [(P["i1"][0], P["dx1"][0], P["i2"][0], P["dx2"][0], P["phi"][0]) for P in Ps]
        if same:
            assert pos[0] == pos[1]
            for c in ("u1", "u2", "u3"):
                assert Ps[1][c][0] == 2.0 * Ps[0][c][0]
        else:
            assert pos[0] != pos[1]


def test_ultrarelativistic_limit_is_massless(O):
    """A massive neutral particle with large |u| moves on the photon's path up
    to O(1/gamma^2) (Sec. 2.3: the mass term is the only difference): the gap
    after 300 steps shrinks a hundredfold when |u| grows tenfold."""
    a = 0.9
    rh = 1 + math.sqrt(1 - a * a)
    prm = params(O, a, 1.0, 0.9 * rh, 40.0, 256, 0.02)
    F = np.zeros((33,) + prm.shape())
    dxi, dth = grid(prm.r_min, prm.r_max, 256, 256)
    gaps = []
    for s in (1e3, 1e4):
        P = single(O, prm, 8.0, 1.0, -0.7 * s, 0.4 * s, 3.0 * s, 7)
        Q = single(O, prm, 8.0, 1.0, -0.7 * s, 0.4 * s, 3.0 * s, 3)
        for _ in range(300):
            O.push(prm, F, P)
            O.push(prm, F, Q)
        rp, tp = position(P, 0, prm.r_min, dxi, dth)
        rq, tq = position(Q, 0, prm.r_min, dxi, dth)
        gaps.append(abs(rp - rq) + rp * abs(tp - tq) + rp * abs(P["phi"][0] - Q["phi"][0]))
    assert gaps[1] < 1e-7
    assert 90.0 < gaps[0] / gaps[1] < 110.0
