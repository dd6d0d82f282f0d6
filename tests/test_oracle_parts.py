"""Pins of the oracle parts that no printed value fixes: the gather's staggering
and axis ghosts (reading R2, R3), the current filter's axis parities (R15), the
placement of the out-of-plane current J^3 (R11) and the outer absorbing layer
(R16).  Each pin is a property the part must have whatever its implementation
(exact reproduction of fields the scheme represents exactly, a moment of the
deposit, stationarity, absorption), and each is shown to fail for a planted
mistake (a patched copy of the oracle, see oracle.planted)."""
import math

import numpy as np
import pytest

from paper_2511_17701_amd.workloads import WORKLOADS

# Yee locations (Sec. 3.3.1) as half-cell offsets (x1, x2): D^1 (i+1/2, j),
# D^2 (i, j+1/2), D^3 (i, j); B^1 (i, j+1/2), B^2 (i+1/2, j), B^3 (i+1/2, j+1/2)
STAG = {0: (1, 0), 1: (0, 1), 2: (0, 0), 3: (0, 1), 4: (1, 0), 5: (1, 1)}
# axis parity of each component: r even, theta and phi odd (R3)
PARITY = {0: 1, 1: -1, 2: -1, 3: 1, 4: -1, 5: -1}


def params(O, n=24, **kw):
    w = WORKLOADS["c1_64"].scaled(n, n)
    prm = O.Params.make(w.a, w.M, w.r_min, w.r_max, n, n, 0.0, **kw)
    prm.dt = O.courant_dt(prm, 0.5)
    return prm


def linear_planes(O, prm, coef, upper):
    """Field set whose six gathered planes (D at 0..2, B^n at 9..11) hold, at
    each component's own staggered points x = (i + o1/2, j + o2/2), the function
    a + b x1 for the even components and (a + b x1) s for the odd ones, with
    s = x2 (lower axis) or n_th - x2 (upper axis): linear in x, with the axis
    parity of the component, so bilinear interpolation must return it exactly
    once the ghost rows are filled by the axis reflection."""
    g, nr, nt = prm.ng, prm.n_r, prm.n_th
    F = np.zeros((33,) + prm.shape())
    for c in range(6):
        o1, o2 = STAG[c]
        x1 = (np.arange(nr + 2 * g) - g + 0.5 * o1)[:, None]
        x2 = (np.arange(nt + 2 * g) - g + 0.5 * o2)[None, :]
        a, b = coef[c]
        val = (a + b * x1) * np.ones_like(x2)
        if PARITY[c] < 0:
            val = val * ((nt - x2) if upper else x2)
        F[(0 if c < 3 else 9) + c % 3] = val
    O.axis_bc(prm, F[0:3], 0)
    O.axis_bc(prm, F[9:12], 1)
    return F


def exact(coef, c, x1, x2, nt, upper):
    a, b = coef[c]
    v = a + b * x1
    return v * ((nt - x2) if upper else x2) if PARITY[c] < 0 else v


def gather_error(O, prm, seed=3):
    """Largest relative error of the gather over random positions in the rows
    next to each axis (where the ghost rows enter) and in the interior."""
    g = np.random.default_rng(seed)
    coef = {c: (g.uniform(0.5, 2.0), g.uniform(-0.1, 0.1)) for c in range(6)}
    nt = prm.n_th
    worst = 0.0
    for upper in (False, True):
        F = linear_planes(O, prm, coef, upper)
        x1s = g.uniform(0.0, prm.n_r - 1e-9, 60)
        near = g.uniform(0.0, 1.0, 60)
        x2s = np.concatenate([near, g.uniform(1.0, nt - 1.0, 20)])
        if upper:
            x2s = nt - x2s
        x2s = np.clip(x2s, 0.0, nt - 1e-12)
        for x1, x2 in zip(np.resize(x1s, len(x2s)), x2s):
            D, B = O.gather(prm, F, x1, x2)
            for c, v in enumerate(np.concatenate([D, B])):
                ref = exact(coef, c, x1, x2, nt, upper)
                worst = max(worst, abs(v - ref) / max(1.0, abs(ref)))
    return worst


def test_gather_reproduces_linear_fields(O):
    """R2 + R3: every one of the six staggered components, filled with a linear
    function of its own code coordinates that has the component's axis parity,
    is returned exactly (to round-off) at random particle positions, also in
    rows 0 and n_th - 1 where the interpolation reads the axis ghost rows and
    in the radial edge cells."""
    assert gather_error(O, params(O)) <= 1e-13


@pytest.mark.parametrize("plant", [
    # B^3 sampled at (i+1/2, j) instead of (i+1/2, j+1/2): a half-cell stagger slip
    ("static const int STAG_B[3][2] = {{0, 1}, {1, 0}, {1, 1}};",
     "static const int STAG_B[3][2] = {{0, 1}, {1, 0}, {1, 0}};"),
    # D^1 sampled at the node instead of the r-edge
    ("static const int STAG_D[3][2] = {{1, 0}, {0, 1}, {0, 0}};",
     "static const int STAG_D[3][2] = {{0, 0}, {0, 1}, {0, 0}};"),
    # phi components even across the axis
    ("const double par[3] = {1.0, -1.0, -1.0};", "const double par[3] = {1.0, -1.0, 1.0};"),
    # the half-cell shift of a staggered component taken the wrong way
    ("if (dx2 >= 0.5) { w2 = dx2 - 0.5; } else { k2 = i2 - 1; w2 = dx2 + 0.5; }",
     "if (dx2 >= 0.5) { w2 = dx2 - 0.5; } else { k2 = i2 - 1; w2 = dx2 - 0.5; }"),
])
def test_gather_pin_fails_planted_mistakes(O, plant):
    with O.planted(plant):
        err = gather_error(O, params(O))
    assert err >= 1e-6, err


# ------------------------------------------------------------- filter

def filter_error(O, prm, seed=4):
    """One to n_f filter passes on current planes that are linear in (x1, x2)
    with the components' axis parities (J^1 even, J^2 and J^3 odd): linear
    functions are fixed points of the (1,2,1)/4 stencil, so the filter must
    leave them unchanged also on the rows whose stencil reads the axis ghosts
    (checked away from the radial edges of the filtered range)."""
    g = np.random.default_rng(seed)
    nr, nt, gg = prm.n_r, prm.n_th, prm.ng
    worst = 0.0
    for upper in (False, True):
        F = np.zeros((33,) + prm.shape())
        coef = [(g.uniform(0.5, 2.0), g.uniform(-0.1, 0.1)) for _ in range(3)]
        ref = []
        for c, (o1, o2) in enumerate(((1, 0), (0, 1), (0, 0))):
            x1 = (np.arange(nr + 2 * gg) - gg + 0.5 * o1)[:, None]
            x2 = (np.arange(nt + 2 * gg) - gg + 0.5 * o2)[None, :]
            v = (coef[c][0] + coef[c][1] * x1) * np.ones_like(x2)
            if c > 0:
                v = v * ((nt - x2) if upper else x2)
            F[18 + c] = v
            ref.append(v.copy())
        O.filter_currents(prm, F)
        rows = slice(gg + nt - 4, gg + nt + 1) if upper else slice(gg, gg + 5)
        cols = slice(gg + prm.n_filter + 1, gg + nr - prm.n_filter - 1)
        for c in range(3):
            d = np.abs(F[18 + c] - ref[c])[cols, rows]
            if c == 1 and upper:
                d = d[:, :-1]   # J^2 has n_th half rows: the last node row is not one of them
            worst = max(worst, d.max() / np.abs(ref[c][cols, rows]).max())
    return worst


def test_filter_keeps_linear_currents_at_the_axes(O):
    """R15 + R3 at the axis: the filter's theta ghosts continue each current
    component with its axis parity, so currents linear in the code coordinates
    with those parities pass n_f = 3 filter passes unchanged on the axis rows
    and the rows next to them."""
    assert filter_error(O, params(O, n_filter=3)) <= 1e-14


@pytest.mark.parametrize("plant", [
    ("const double par[3] = {1.0, -1.0, -1.0};", "const double par[3] = {-1.0, -1.0, -1.0};"),
    ("const double par[3] = {1.0, -1.0, -1.0};", "const double par[3] = {1.0, 1.0, -1.0};"),
    ("const double par[3] = {1.0, -1.0, -1.0};", "const double par[3] = {1.0, -1.0, 1.0};"),
    # ghosts of a staggered component mirrored about the wrong row
    ("C[IX(p, i, -g)] = par[comp] * C[IX(p, i, g - 1)];", "C[IX(p, i, -g)] = par[comp] * C[IX(p, i, g)];"),
])
def test_filter_pin_fails_planted_mistakes(O, plant):
    with O.planted(plant):
        err = filter_error(O, params(O, n_filter=3))
    assert err >= 1e-3, err


# ------------------------------------------------------------- J^3 placement

def j3_moments(O, prm, seed=5):
    """Single charged particles away from the axis rows: their J^3 nodes
    carry weights whose first moment is the midpoint of the particle's path
    (reading R11: the shape at the path midpoint), for each of many paths.
    Returns the largest distance between the weighted mean node and the
    midpoint, in cells."""
    g = np.random.default_rng(seed)
    F = O.fields_init_wald(prm, 1.0)
    n = 40
    P = O.particles_init(prm, n // 2, 0, 1.0, 0, 7)
    P["i1"][:] = g.integers(3, prm.n_r - 4, n).astype(np.int32)
    P["i2"][:] = g.integers(3, prm.n_th - 4, n).astype(np.int32)
    P["dx1"][:] = g.uniform(0, 1, n)
    P["dx2"][:] = g.uniform(0, 1, n)
    P["tag"][:] = np.where(np.arange(n) % 2 == 0, 1, 2).astype(np.uint8)
    O.push(prm, F, P)   # saves the previous position, then moves
    gg = prm.ng
    worst = 0.0
    for k in range(n):
        one = {key: v[k:k + 1].copy() for key, v in P.items()}
        Fk = np.zeros_like(F)
        O.deposit(prm, Fk, one)
        J3 = Fk[20]
        tot = J3.sum()
        ii, jj = np.meshgrid(np.arange(J3.shape[0]) - gg, np.arange(J3.shape[1]) - gg, indexing="ij")
        m1, m2 = (ii * J3).sum() / tot, (jj * J3).sum() / tot
        xa = (one["i1p"][0] + one["dx1p"][0], one["i2p"][0] + one["dx2p"][0])
        xb = (one["i1"][0] + one["dx1"][0], one["i2"][0] + one["dx2"][0])
        mid = (0.5 * (xa[0] + xb[0]), 0.5 * (xa[1] + xb[1]))
        worst = max(worst, abs(m1 - mid[0]), abs(m2 - mid[1]))
    return worst


def test_j3_first_moment_is_the_path_midpoint(O):
    """R11: the first moment of a particle's J^3 node weights is the midpoint
    of its path (the second and the zeroth moment are fixed by other pins)."""
    assert j3_moments(O, params(O, charge_scale=1.0)) <= 1e-12


@pytest.mark.parametrize("plant", [
    # J^3 placed at the start point of the path
    ("double xm = 0.5 * (xa + xb), ym = 0.5 * (ya + yb);\n  orc_metric m;",
     "double xm = xa, ym = ya;\n  orc_metric m;"),
    # J^3 placed at the end point
    ("double xm = 0.5 * (xa + xb), ym = 0.5 * (ya + yb);\n  orc_metric m;",
     "double xm = xb, ym = yb;\n  orc_metric m;"),
])
def test_j3_pin_fails_planted_mistakes(O, plant):
    with O.planted(plant):
        d = j3_moments(O, params(O, charge_scale=1.0))
    assert d >= 1e-4, d


# ------------------------------------------------------------- absorbing layer

def wald_layer_deviation(O, n, n_absorb, T=4.0):
    """Wald vacuum (a stationary solution, B0 = 1, the C1 geometry on an n^2
    grid) evolved by the field stages for a time T: largest relative deviation
    from the initial data over the six components, on the outer n/4 columns
    (the layer when n_absorb = n/4) and in the interior r in [6, 12] before
    them."""
    w = WORKLOADS["c1_64"].scaled(n, n)
    prm = O.Params.make(w.a, w.M, w.r_min, w.r_max, n, n, 0.0, n_absorb=n_absorb)
    prm.dt = O.courant_dt(prm, 0.5)
    F = O.fields_init_wald(prm, 1.0)
    F0 = F.copy()
    for _ in range(int(round(T / prm.dt))):
        O.field_advance(prm, F, 0)
        O.field_advance(prm, F, 1)
    g = prm.ng
    dxi = math.log(prm.r_max / prm.r_min) / n
    r = prm.r_min * np.exp((np.arange(n + 2 * g) - g) * dxi)
    i = np.arange(n + 2 * g) - g
    layer = (i >= n - n // 4) & (i < n)
    inner = (r > 6.0) & (r < 12.0) & (i < n - n // 4)
    return [max(np.abs(F[c] - F0[c])[sel][:, g:g + n].max() /
                np.abs(F0[c][sel][:, g:g + n]).max() for c in range(6)) for sel in (layer, inner)]


def test_absorbing_layer_keeps_the_stationary_state(O):
    """R16: the layer relaxes towards the initial (stationary) fields, so the
    Wald vacuum stays stationary inside the layer up to truncation error that
    falls at second order (at least 3x from 32^2 to 64^2), and the interior
    before the layer evolves as without it (Sec. 3.3.3: matched to the
    initial values)."""
    lay32, _ = wald_layer_deviation(O, 32, 8)
    lay64, in64 = wald_layer_deviation(O, 64, 16)
    _, in64_bare = wald_layer_deviation(O, 64, 0)
    assert lay64 <= 5e-2 and lay32 / lay64 >= 3.0, (lay32, lay64)
    assert in64 <= 1.01 * in64_bare + 1e-12, (in64, in64_bare)


def test_absorbing_layer_stationary_pin_fails_planted_mistakes(O):
    """Relaxing towards zero, or away from the initial fields, breaks the pin."""
    for plant in (("C[o] = C[o] - lam * (C[o] - C0[o]);", "C[o] = C[o] - lam * C[o];"),
                  ("C[o] = C[o] - lam * (C[o] - C0[o]);", "C[o] = C[o] + lam * (C[o] - C0[o]);")):
        with O.planted(plant):
            lay64, _ = wald_layer_deviation(O, 64, 16)
        assert lay64 > 5e-2, (plant, lay64)


def reflected_pulse(O, n_absorb, n_r=64, n_th=8, r_max=30.0):
    """A toroidal magnetic pulse (B^3 ~ exp(-(r - 10)^2 / 4.5) / r, no
    background) around a Schwarzschild hole (a = 0, inner edge 0.9 r_h inside
    the horizon, which absorbs what falls in): the part running outwards meets
    the outer boundary at r_max and, unless absorbed there, returns.  Returns
    the largest |D^1|, |D^2|, |B^3| left in r in [4, 18] at t in [56, 66], when
    the returning part crosses that window (the initial pulse has left it by
    then)."""
    prm = O.Params.make(0.0, 1.0, 1.8, r_max, n_r, n_th, 0.0, n_absorb=n_absorb)
    prm.dt = O.courant_dt(prm, 0.5)
    g = prm.ng
    dxi = math.log(prm.r_max / prm.r_min) / n_r
    r = prm.r_min * np.exp((np.arange(n_r + 2 * g) - g + 0.5) * dxi)
    F = O.fields_init_wald(prm, 0.0)          # zero fields, zero layer targets
    prof = (np.exp(-(r - 10.0) ** 2 / 4.5) / r)[:, None] * np.ones(n_th + 2 * g)[None, :]
    F[5] += prof
    F[11] += prof
    win = (r > 4.0) & (r < 18.0)
    late = np.zeros(3)
    for s in range(int(round(66.0 / prm.dt))):
        O.field_advance(prm, F, 0)
        O.field_advance(prm, F, 1)
        if (s + 1) * prm.dt >= 56.0:
            m = np.abs(F[[0, 1, 5]][:, win][:, :, g:g + n_th]).max(axis=(1, 2))
            late = np.maximum(late, m)
    return late


def test_absorbing_layer_absorbs_an_outgoing_pulse(O):
    """R16: with a 16-cell layer the pulse that returns from the outer boundary
    is at least 10x weaker in every component it excites than without it."""
    bare = reflected_pulse(O, 0)
    layer = reflected_pulse(O, 16)
    assert np.all(bare >= 10.0 * layer), (bare, layer)


def test_absorbing_layer_absorption_pin_fails_planted_mistake(O):
    """A layer placed past the outer edge of the grid (its start taken at
    n_r + n_absorb instead of n_r - n_absorb) fails the absorption pin."""
    bare = reflected_pulse(O, 0)
    with O.planted(("double x0 = (double)(p->n_r - p->n_absorb);", "double x0 = (double)(p->n_r + p->n_absorb);")):
        layer = reflected_pulse(O, 16)
    assert not np.all(bare >= 10.0 * layer), (bare, layer)


def test_absorbing_ramp_shape(O):
    """R16's ramp: lambda is 0 up to the layer's inner edge x0 = n_r - n_absorb,
    grows monotonically to 1 at the outer edge and stays 1 beyond it, and
    starts with zero slope and curvature (a smooth onset reflects nothing at
    the edge to second order: finite differences of lambda at x0 vanish like
    h^3)."""
    prm = O.Params.make(0.9, 1.0, 1.3, 20.0, 64, 32, 0.01, n_absorb=16)
    x0, xe = 64 - 16, 64.0
    xs = np.linspace(0.0, 70.0, 7001)
    lam = np.array([O.match_lambda(prm, x) for x in xs])
    assert (lam[xs <= x0] == 0.0).all()
    assert (lam[xs >= xe] == 1.0).all()
    assert (np.diff(lam) >= 0.0).all()
    assert ((lam > 0) & (lam < 1))[(xs > x0) & (xs < xe)].all()
    h = np.array([1e-1, 1e-2])
    vals = np.array([O.match_lambda(prm, x0 + d) for d in h])
    assert vals[0] / vals[1] == pytest.approx(1e3, rel=1e-6)    # ~ h^3 at the onset
    bare = O.Params.make(0.9, 1.0, 1.3, 20.0, 64, 32, 0.01, n_absorb=0)
    assert all(O.match_lambda(bare, x) == 0.0 for x in (0.0, 40.0, 63.9, 64.0, 70.0))
