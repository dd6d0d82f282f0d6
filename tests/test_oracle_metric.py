"""Pins of the oracle's metric, derivatives and tetrads against what the paper
and the mathematics fix (no GPU)."""
import json
import math
import os

import numpy as np
import pytest
import sympy as sp

from _helpers import bl_energy, grid, single

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1.json")


def params(O, a=0.9, M=1.0, r_min=1.0, r_max=20.0, n=64, dt=0.01):
    return O.Params.make(a, M, r_min, r_max, n, n, dt)


def rows():
    with open(GOLD) as f:
        return json.load(f)["rows"]


def decimals(x):
    t = repr(float(x))
    return len(t.split(".")[1]) if "." in t else 0


def theta_of(s):
    return {"pi/2": math.pi / 2, "pi/2-0.2": math.pi / 2 - 0.2}[s]


# --------------------------------------------------------------- Table 1

@pytest.mark.parametrize("row", rows(), ids=lambda r: r["name"])
def test_table1_energy_and_momentum(O, row):
    """E = alpha gamma - beta^1 u_1 - (q/m) A_0 and L = u_3 + (q/m) A_3 of the
    printed initial data reproduce Table 1 to the printed digits."""
    a, M = row["a"], row["M"]
    rh = M + math.sqrt(M * M - a * a) if M > 0 else 1.0
    prm = params(O, a=a, M=M, r_min=0.9 * rh, r_max=row["r_max"], n=row["N"], dt=row["dt"])
    tag = {"neutral": 3, "positron": 1}[row["species"]]
    P = single(O, prm, row["r"], theta_of(row["theta"]), row["u1"], 0.0, row["u3"], tag)
    E, L = O.energy_momentum(prm, P, row["B0"])
    # half a unit of the last printed digit, plus the effect of rounded inputs
    tol = 0.5 * 10.0 ** -decimals(row["E"]) + 1e-4 * abs(row["E"])
    assert abs(E[0] - row["E"]) <= tol, (E[0], row["E"])
    if row["name"] == "SR-EM":
        # the printed L of this row equals the mechanical u_3 (canonical: u_3 + A_3 = 35)
        assert L[0] == pytest.approx(row["u3"] + 0.5 * row["B0"] * row["r"] ** 2)
    else:
        assert abs(L[0] - row["L"]) <= 1e-5 * abs(row["L"]) + 5e-4, (L[0], row["L"])


@pytest.mark.parametrize("name", ["GR", "GR-EM-2D"])
def test_table1_bl_initial_data(O, name):
    """u_1(KS) from the BL-KS transformation at BL turning point and E from the
    BL normalisation reproduce the printed E, u_1; the oracle's KS energy of that
    state equals the BL energy to round-off (independent metric check)."""
    row = [r for r in rows() if r["name"] == name][0]
    a, M, r, th = row["a"], row["M"], row["r"], theta_of(row["theta"])
    u3 = row["u3"]
    E_bl, u_r = bl_energy(a, M, r, th, u3)
    assert abs(E_bl - row["E"]) < 6e-4 * row["E"]
    assert abs(u_r - row["u1"]) < 1e-3 * abs(row["u1"]) + 1e-5
    prm = params(O, a=a, M=M, r_min=0.9 * (M + math.sqrt(M * M - a * a)), r_max=row["r_max"],
                 n=row["N"])
    P = single(O, prm, r, th, u_r, 0.0, u3, 3)
    E, _ = O.energy_momentum(prm, P, 0.0)
    assert E[0] == pytest.approx(E_bl, rel=1e-13)


def test_bl_energy_random(O):
    """KS energy of BL turning-point states equals the BL energy for random
    spins, radii, polar angles and angular momenta (metric vs textbook BL)."""
    g = np.random.default_rng(1)
    for _ in range(40):
        a = g.uniform(0, 0.999)
        r = g.uniform(2.5, 30)
        th = g.uniform(0.2, math.pi - 0.2)
        L = g.uniform(-4, 4)
        prm = params(O, a=a, r_min=0.9 * (1 + math.sqrt(1 - a * a)), r_max=40.0, n=128)
        E_bl, u_r = bl_energy(a, 1.0, r, th, L)
        P = single(O, prm, r, th, u_r, 0.0, L, 3)
        E, _ = O.energy_momentum(prm, P, 0.0)
        assert E[0] == pytest.approx(E_bl, rel=2e-13)


# ----------------------------------------------------- 4-metric, identities

def printed_metric(a, M, r, th):
    """App. A covariant and contravariant Kerr-Schild metric (2r -> 2Mr)."""
    s, c = math.sin(th), math.cos(th)
    Sig = r * r + a * a * c * c
    Del = r * r - 2 * M * r + a * a
    A = (r * r + a * a) ** 2 - a * a * Del * s * s
    z = 2 * M * r / Sig
    g = np.array([[-(1 - z), z, 0, -a * z * s * s],
                  [z, 1 + z, 0, -a * (1 + z) * s * s],
                  [0, 0, Sig, 0],
                  [-a * z * s * s, -a * (1 + z) * s * s, 0, A * s * s / Sig]])
    gi = np.array([[-(1 + z), z, 0, 0],
                   [z, Del / Sig, 0, a / Sig],
                   [0, 0, 1 / Sig, 0],
                   [0, a / Sig, 0, 1 / (Sig * s * s)]])
    return g, gi


@pytest.mark.parametrize("M", [1.0, 0.7, 0.0])
def test_four_metric_from_3p1(O, M):
    """The 4-metric assembled from the oracle's lapse, shift and spatial metric
    equals the printed Kerr-Schild g_{mu nu} and g^{mu nu}; h^ij h_jk = delta,
    det h = (sqrt h)^2, beta_i beta^i = z^2/(1+z)."""
    g = np.random.default_rng(2)
    for _ in range(20):
        a = g.uniform(0, 0.99) if M > 0 else 0.0
        prm = params(O, a=a, M=M, r_min=1.1, r_max=25.0, n=96)
        dxi, dth = grid(prm.r_min, prm.r_max, prm.n_r, prm.n_th)
        x1, x2 = g.uniform(0, 96), g.uniform(1, 95)
        m = O.metric_at(prm, x1, x2, clamp=False)
        r, th, R = m["r"], m["th"], m["R"]
        hu = np.array([[m["hu11"] * R * R, 0, m["hu13"] * R], [0, m["hu22"] * dth * dth, 0],
                       [m["hu13"] * R, 0, m["hu33"]]])
        hl = np.array([[m["hl11"] / R ** 2, 0, m["hl13"] / R], [0, m["hl22"] / dth ** 2, 0],
                       [m["hl13"] / R, 0, m["hl33"]]])
        al, beta = m["alpha"], np.array([m["beta1"] * R, 0, 0])
        gi = np.zeros((4, 4))
        gi[0, 0] = -1 / al ** 2
        gi[0, 1:] = gi[1:, 0] = beta / al ** 2
        gi[1:, 1:] = hu - np.outer(beta, beta) / al ** 2
        bl = hl @ beta
        gl = np.zeros((4, 4))
        gl[0, 0] = -al ** 2 + bl @ beta
        gl[0, 1:] = gl[1:, 0] = bl
        gl[1:, 1:] = hl
        G, GI = printed_metric(a, M, r, th)
        np.testing.assert_allclose(gl, G, rtol=1e-13, atol=1e-13 * np.abs(G).max())
        np.testing.assert_allclose(gi, GI, rtol=1e-13, atol=1e-13 * np.abs(GI).max())
        np.testing.assert_allclose(hu @ hl, np.eye(3), atol=1e-13)
        sqrt_h_phys = m["sqrt_h"] / (R * dth)
        assert np.linalg.det(hl) == pytest.approx(sqrt_h_phys ** 2, rel=1e-12)
        z = 2 * M * r / m["Sig"]
        assert bl @ beta == pytest.approx(z * z / (1 + z), rel=1e-12, abs=1e-15)


def test_flat_reduction(O):
    """M = 0, a = 0 gives the spherical Minkowski metric of App. A
    (kerr_schild_0) with dr -> dxi r on the log grid: alpha = 1, beta = 0,
    h_ij = diag(R^2, dth^2 r^2, r^2 sin^2), sqrt(h) = R dth r^2 sin, and the
    printed derivatives d_r h^22, d_r h^33, d_th h^33."""
    prm = params(O, a=0.0, M=0.0, r_min=0.5, r_max=30.0, n=80)
    dxi, dth = grid(prm.r_min, prm.r_max, 80, 80)
    for x1, x2 in [(3.3, 17.6), (40.2, 40.0), (71.9, 2.2)]:
        m = O.metric_at(prm, x1, x2, clamp=False)
        r, s, c, R = m["r"], m["s"], m["c"], m["R"]
        assert m["alpha"] == 1.0 and m["beta1"] == 0.0 and m["hu13"] == 0.0
        assert m["hl11"] == pytest.approx(R * R, rel=1e-15)
        assert m["hl22"] == pytest.approx(dth * dth * r * r, rel=1e-15)
        assert m["hl33"] == pytest.approx(r * r * s * s, rel=1e-15)
        assert m["sqrt_h"] == pytest.approx(R * dth * r * r * s, rel=1e-14)
        assert m["d_hu22"][0] == pytest.approx(-R * 2 / (r ** 3 * dth ** 2), rel=1e-13)
        assert m["d_hu33"][0] == pytest.approx(-R * 2 / (r ** 3 * s * s), rel=1e-13)
        assert m["d_hu33"][1] == pytest.approx(-2 * dth * c / (r * r * s ** 3), rel=1e-13)
        assert m["d_alpha"] == (0.0, 0.0) and m["d_beta1"] == (0.0, 0.0)
        assert m["d_hu13"] == (0.0, 0.0) and m["d_hu22"][1] == 0.0


# ------------------------------------------------------------- derivatives

def _symbolic_coeffs():
    """alpha, beta^1, h^11, h^22, h^33, h^13 in code components as sympy
    expressions of (x1, x2), derived from the printed contravariant 4-metric:
    alpha^2 = -1/g^00, beta^i = -g^0i/g^00, h^ij = g^ij - g^0i g^0j / g^00."""
    x1, x2, a, M, xi0, dxi, dth = sp.symbols("x1 x2 a M xi0 dxi dth", real=True)
    r = sp.exp(xi0 + x1 * dxi)
    th = x2 * dth
    Sig = r ** 2 + a ** 2 * sp.cos(th) ** 2
    Del = r ** 2 - 2 * M * r + a ** 2
    z = 2 * M * r / Sig
    g00, g01, g11, g13 = -(1 + z), z, Del / Sig, a / Sig
    g22, g33 = 1 / Sig, 1 / (Sig * sp.sin(th) ** 2)
    R = dxi * r
    alpha = sp.sqrt(-1 / g00)
    beta1 = (-g01 / g00) / R
    h11 = (g11 - g01 * g01 / g00) / R ** 2
    h13 = g13 / R
    h22 = g22 / dth ** 2
    h33 = g33
    syms = (x1, x2, a, M, xi0, dxi, dth)
    out = {}
    for name, ex in [("alpha", alpha), ("beta1", beta1), ("hu11", h11), ("hu22", h22),
                     ("hu33", h33), ("hu13", h13)]:
        out[name] = [sp.lambdify(syms, ex, "mpmath"),
                     sp.lambdify(syms, sp.diff(ex, x1), "mpmath"),
                     sp.lambdify(syms, sp.diff(ex, x2), "mpmath")]
    return out


def test_derivatives_vs_symbolic(O):
    """The twelve metric derivatives used by the momentum iteration equal the
    symbolic derivatives (sympy, 30-digit evaluation) of coefficients derived
    from the printed inverse 4-metric (App. A), for M = 1 and M != 1."""
    import mpmath
    mpmath.mp.dps = 30
    f = _symbolic_coeffs()
    g = np.random.default_rng(3)
    for M in (1.0, 0.6):
        for _ in range(12):
            a = g.uniform(0, 0.99)
            prm = params(O, a=a, M=M, r_min=0.9, r_max=40.0, n=128)
            dxi, dth = grid(prm.r_min, prm.r_max, 128, 128)
            x1, x2 = g.uniform(0, 128), g.uniform(0.5, 127.5)
            m = O.metric_at(prm, x1, x2, clamp=False)
            args = (x1, x2, a, M, math.log(prm.r_min), dxi, dth)
            for name, dname in [("alpha", "d_alpha"), ("beta1", "d_beta1"), ("hu11", "d_hu11"),
                                ("hu22", "d_hu22"), ("hu33", "d_hu33"), ("hu13", "d_hu13")]:
                val = float(f[name][0](*args))
                assert m[name] == pytest.approx(val, rel=1e-13, abs=1e-300)
                for k in range(2):
                    ref = float(f[name][1 + k](*args))
                    scale = abs(val) * 1e-12 + abs(ref) * 1e-11 + 1e-300
                    assert abs(m[dname][k] - ref) <= scale, (M, name, k, m[dname][k], ref)


# ------------------------------------------------------------------ tetrads

def test_tetrad_orthonormal_and_inverse(O):
    """Tetrad transforms built from the App. A matrices: norms are preserved
    (|u_hat|^2 = h^ij u_i u_j, |A_hat|^2 = h_ij A^i A^j), the pairing A^i u_i is
    invariant, and each inverse undoes its forward map."""
    g = np.random.default_rng(4)
    for _ in range(30):
        a = g.uniform(0, 0.99)
        prm = params(O, a=a, r_min=1.0, r_max=30.0, n=64)
        x1, x2 = g.uniform(0, 64), g.uniform(0.05, 63.95)
        m = O.metric_at(prm, x1, x2, clamp=False)
        hu = np.array([[m["hu11"], 0, m["hu13"]], [0, m["hu22"], 0], [m["hu13"], 0, m["hu33"]]])
        hl = np.array([[m["hl11"], 0, m["hl13"]], [0, m["hl22"], 0], [m["hl13"], 0, m["hl33"]]])
        u = g.normal(size=3) * np.array([m["R"], 1e-2, 3.0])
        A = g.normal(size=3) / np.array([m["R"], 1e-2, 3.0])
        uh = O.tetrad(prm, x1, x2, "cov_to_hat", u, clamp=False)
        Ah = O.tetrad(prm, x1, x2, "con_to_hat", A, clamp=False)
        assert uh @ uh == pytest.approx(u @ hu @ u, rel=1e-13)
        assert Ah @ Ah == pytest.approx(A @ hl @ A, rel=1e-13)
        assert uh @ Ah == pytest.approx(u @ A, rel=1e-12, abs=1e-14 * abs(u) @ abs(A))
        np.testing.assert_allclose(O.tetrad(prm, x1, x2, "hat_to_cov", uh, clamp=False), u,
                                   rtol=1e-13, atol=1e-14 * np.abs(u).max())
        np.testing.assert_allclose(O.tetrad(prm, x1, x2, "hat_to_con", Ah, clamp=False), A,
                                   rtol=1e-13, atol=1e-14 * np.abs(A).max())
