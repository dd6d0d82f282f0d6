"""Reference gradient of the frozen-field particle update (test infrastructure).

Only `tests/` may use this module; the product path never imports it.

A plain PyTorch-CPU, FP64 restatement of the particle update of Sec. 3.1
(steps 2-10) with the particle boundaries of Sec. 3.3.3, in a frozen field
F = B0 * F1 (the Wald field of eq. Wald is linear in its amplitude), written
for automatic differentiation:

  - the metric of App. A is written out from its closed forms (Sigma, Delta,
    A, z, lapse, shift, h^ij, h_ij and the tetrad factors of the App. A
    matrices); its first derivatives, which drive the momentum equation, are
    taken by torch.autograd with create_graph, so the gradient of the step
    sees second derivatives of the metric without any hand-derived formula;
  - the two implicit-midpoint iterations (eq. discretized-geodesic-u and
    eq. discretized-geodesic-x) run their fixed number of iterations, or stop
    once every iterate repeats exactly (the fixed point: the same values as
    further iterations), and are differentiated unrolled, which is the exact
    derivative of the discrete map (and equals the implicit-function-theorem
    derivative once the iterations have converged);
  - positions are (int cell, FP64 offset) pairs as in the C oracle; the
    integer shift of a renormalisation carries no derivative;
  - the polar angle is clamped at small_angle in metric evaluations (a
    clamped angle has zero derivative).

Readings shared with the C oracle: R2 (bilinear gather from the staggered
locations), R4, R5, R6, R7, R10, R12, R22, R27 (a particle that leaves is
frozen at its last position; the C oracle empties it on the next push).

The forward map is pinned to the C oracle's push (tests/test_oracle_adjoint.py),
its derivatives to central differences of the C oracle.
"""
from __future__ import annotations

import math

import torch

DT = torch.float64


def _grid(p):
    """log spacing of r - r0 and the uniform spacing of eta (App. A map)."""
    r0 = getattr(p, "r0", 0.0)
    dxi = math.log((p.r_max - r0) / (p.r_min - r0)) / p.n_r
    deta = math.pi / p.n_th
    return dxi, deta


def metric(p, x1, x2):
    """Lapse, shift, inverse and lower spatial metric in code components at
    code position (x1, x2) (App. A, quasi-spherical map: r = r0 + exp(xi),
    theta(eta) with concentration h0; index 1 carries R = dr/dx1, index 2
    carries T = dtheta/dx2).  Beyond either axis (a midpoint of the
    coordinate iteration can fall there) the polar map is continued by
    reflection, theta(-x2) = -theta(x2), theta(2 n_th - x2) = 2 pi - theta(x2),
    as in the C oracle (reading R23)."""
    dxi, deta = _grid(p)
    a, M = p.a, p.M
    r0, h0 = getattr(p, "r0", 0.0), getattr(p, "h0", 0.0)
    e = torch.exp(math.log(p.r_min - r0) + x1 * dxi)
    r = r0 + e
    R = dxi * e
    lo, hi = x2 < 0.0, x2 > p.n_th
    xr = torch.where(lo, -x2, torch.where(hi, 2.0 * p.n_th - x2, x2))
    eta = xr * deta
    y = eta / math.pi
    th = eta + 2.0 * h0 * eta * (math.pi - 2.0 * eta) * (math.pi - eta) / (math.pi * math.pi)
    th = torch.where(lo, -th, torch.where(hi, 2.0 * math.pi - th, th))
    T = deta * (1.0 + 2.0 * h0 + 12.0 * h0 * y * (y - 1.0))
    th = torch.clamp(th, p.small_angle, math.pi - p.small_angle)
    s, c = torch.sin(th), torch.cos(th)
    Sig = r * r + a * a * c * c
    Del = r * r - 2.0 * M * r + a * a
    A = (r * r + a * a) ** 2 - a * a * Del * s * s
    z = 2.0 * M * r / Sig
    m = {}
    m["alpha"] = 1.0 / torch.sqrt(1.0 + z)
    m["beta1"] = z / (1.0 + z) / R
    m["hu11"] = A / (Sig * (Sig + 2.0 * M * r)) / (R * R)
    m["hu13"] = a / Sig / R
    m["hu22"] = 1.0 / Sig / (T * T)
    m["hu33"] = 1.0 / (Sig * s * s)
    hl13 = -a * (1.0 + z) * s * s * R
    hl22 = Sig * T * T
    hl33 = A * s * s / Sig
    # tetrad factors of the App. A matrices (reading R22)
    m["s11"] = torch.sqrt(m["hu11"])
    m["s22"] = torch.sqrt(hl22)
    m["s33"] = torch.sqrt(hl33)
    m["k13"] = hl13 / hl33
    return m


def metric_with_derivatives(p, x1, x2):
    """metric() plus d/dx1, d/dx2 of alpha, beta^1 and h^ij (by autograd,
    kept in the graph so that their own derivatives are available)."""
    if not x1.requires_grad:
        x1 = x1.clone().requires_grad_(True)
    if not x2.requires_grad:
        x2 = x2.clone().requires_grad_(True)
    m = metric(p, x1, x2)
    for k in ("alpha", "beta1", "hu11", "hu22", "hu33", "hu13"):
        g1, g2 = torch.autograd.grad(m[k].sum(), (x1, x2), create_graph=True)
        m["d" + k] = (g1, g2)
    return m


def gamma(m, u1, u2, u3, m2=1.0):
    """u^0 alpha = sqrt(m^2 + h^ij u_i u_j) per unit mass (Sec. 2.3); m2 = 0
    for massless particles."""
    return torch.sqrt(m2 + m["hu11"] * u1 * u1 + m["hu22"] * u2 * u2 + m["hu33"] * u3 * u3 +
                      2.0 * m["hu13"] * u1 * u3)


# Yee locations (Sec. 3.3.1): D^1 (i+1/2, j), D^2 (i, j+1/2), D^3 (i, j),
# B^1 (i, j+1/2), B^2 (i+1/2, j), B^3 (i+1/2, j+1/2).
STAG_D = ((1, 0), (0, 1), (0, 0))
STAG_B = ((0, 1), (1, 0), (1, 1))


def interp(p, plane, i1, dx1, i2, dx2, o1, o2):
    """Bilinear interpolation (reading R2) of a plane staggered by half a cell
    in x1 (o1) and/or x2 (o2); `plane` holds the ghost rows."""
    ng = p.ng
    ld = p.n_th + 2 * ng
    k1, w1 = i1, dx1
    if o1:
        hi = dx1 >= 0.5
        k1 = torch.where(hi, i1, i1 - 1)
        w1 = torch.where(hi, dx1 - 0.5, dx1 + 0.5)
    k2, w2 = i2, dx2
    if o2:
        hi = dx2 >= 0.5
        k2 = torch.where(hi, i2, i2 - 1)
        w2 = torch.where(hi, dx2 - 0.5, dx2 + 0.5)
    flat = plane.reshape(-1)

    def at(a, b):
        return flat[(a + ng) * ld + (b + ng)]
    return ((1 - w1) * (1 - w2) * at(k1, k2) + w1 * (1 - w2) * at(k1 + 1, k2) +
            (1 - w1) * w2 * at(k1, k2 + 1) + w1 * w2 * at(k1 + 1, k2 + 1))


def boris(u, E, B, qm, tau):
    """Textbook relativistic Boris step (reading R10) on tetrad components."""
    k = 0.5 * qm * tau
    um = [u[c] + k * E[c] for c in range(3)]
    g = torch.sqrt(1.0 + um[0] ** 2 + um[1] ** 2 + um[2] ** 2)
    t = [k * B[c] / g for c in range(3)]
    t2 = t[0] ** 2 + t[1] ** 2 + t[2] ** 2
    sv = [2.0 * t[c] / (1.0 + t2) for c in range(3)]
    up = [um[0] + (um[1] * t[2] - um[2] * t[1]),
          um[1] + (um[2] * t[0] - um[0] * t[2]),
          um[2] + (um[0] * t[1] - um[1] * t[0])]
    uq = [um[0] + (up[1] * sv[2] - up[2] * sv[1]),
          um[1] + (up[2] * sv[0] - up[0] * sv[2]),
          um[2] + (up[0] * sv[1] - up[1] * sv[0])]
    return [uq[c] + k * E[c] for c in range(3)]


def em_half(p, m, Dc, Bc, qm, u):
    """EM half step (Sec. 3.1 steps 3-5 / 7-9): contravariant D, B and covariant
    u to the tetrad frame, Boris over dt/2 with the lapse-scaled fields, back."""
    s11, s22, s33, k13, al = m["s11"], m["s22"], m["s33"], m["k13"], m["alpha"]
    Dh = [Dc[0] / s11, s22 * Dc[1], k13 * s33 * Dc[0] + s33 * Dc[2]]
    Bh = [Bc[0] / s11, s22 * Bc[1], k13 * s33 * Bc[0] + s33 * Bc[2]]
    uh = [s11 * u[0] - s11 * k13 * u[2], u[1] / s22, u[2] / s33]
    uh = boris(uh, [al * d for d in Dh], [al * b for b in Bh], qm, 0.5 * p.dt)
    return [uh[0] / s11 + k13 * s33 * uh[2], s22 * uh[1], s33 * uh[2]]


def geodesic_momentum(p, m, u, m2=1.0):
    """eq. discretized-geodesic-u: n_iter fixed-point iterations on u_1, u_2
    at fixed x^n with contravariant metric derivatives (R5); u_3 unchanged."""
    us1, us2, u3 = u
    ut1, ut2 = us1, us2
    for _ in range(p.n_iter):
        ub1, ub2 = 0.5 * (us1 + ut1), 0.5 * (us2 + ut2)
        gb = gamma(m, ub1, ub2, u3, m2)
        f = []
        for i in range(2):
            quad = (m["dhu11"][i] * ub1 * ub1 + m["dhu22"][i] * ub2 * ub2 +
                    m["dhu33"][i] * u3 * u3 + 2.0 * m["dhu13"][i] * ub1 * u3)
            f.append(-gb * m["dalpha"][i] + ub1 * m["dbeta1"][i] - m["alpha"] / (2.0 * gb) * quad)
        n1, n2 = us1 + p.dt * f[0], us2 + p.dt * f[1]
        done = torch.equal(n1, ut1) and torch.equal(n2, ut2)
        ut1, ut2 = n1, n2
        if done:   # every iterate repeats: the fixed point (same values as more iterations)
            break
    return [ut1, ut2, u3]


def velocity(m, u, m2=1.0):
    """dx^i/dt = alpha h^ij u_j / gamma - beta^i (i = 1, 2)."""
    iu0 = m["alpha"] / gamma(m, *u, m2)
    return ((m["hu11"] * u[0] + m["hu13"] * u[2]) * iu0 - m["beta1"], m["hu22"] * u[1] * iu0)


def _renorm(i, dx):
    f = torch.floor(dx.detach())
    i = i + f.to(i.dtype)
    dx = dx - f
    over = dx.detach() >= 1.0
    return torch.where(over, i + 1, i), torch.where(over, dx - 1.0, dx)


def step(p, F1, B0, st):
    """One frozen-field particle update.  st: dict of tensors i1, i2 (int64),
    dx1, dx2, u1, u2, u3 (float64), qm (float64 +-1 or 0), m2 (float64 squared
    rest mass, 1 or 0 for massless neutral particles), live (bool).
    F1: (n_planes, n_r + 2 ng, n_th + 2 ng) unit-amplitude field (planes
    D = 0..2 and B = 9..11, the B^n the push reads); B0: amplitude."""
    i1, i2, dx1, dx2 = st["i1"], st["i2"], st["dx1"], st["dx2"]
    u = [st["u1"], st["u2"], st["u3"]]
    qm, live = st["qm"], st["live"]
    m2 = st.get("m2", 1.0)
    x1 = i1.to(DT) + dx1
    x2 = i2.to(DT) + dx2
    m = metric_with_derivatives(p, x1, x2)
    charged = qm != 0.0
    if bool(charged.any()):
        Dc = [B0 * interp(p, F1[c], i1, dx1, i2, dx2, *STAG_D[c]) for c in range(3)]
        Bc = [B0 * interp(p, F1[9 + c], i1, dx1, i2, dx2, *STAG_B[c]) for c in range(3)]
        ue = em_half(p, m, Dc, Bc, qm, u)
        ue = geodesic_momentum(p, m, ue)
        ue = em_half(p, m, Dc, Bc, qm, ue)
        un = geodesic_momentum(p, m, u, m2)
        u = [torch.where(charged, a, b) for a, b in zip(ue, un)]
    else:
        u = geodesic_momentum(p, m, u, m2)
    d1 = torch.zeros_like(dx1)
    d2 = torch.zeros_like(dx2)
    for _ in range(p.n_iter):
        mb = metric(p, x1 + 0.5 * d1, x2 + 0.5 * d2)
        v1, v2 = velocity(mb, u, m2)
        n1, n2 = p.dt * v1, p.dt * v2
        done = torch.equal(n1, d1) and torch.equal(n2, d2)
        d1, d2 = n1, n2
        if done:
            break
    n1, ndx1 = _renorm(i1, dx1 + d1)
    n2, ndx2 = _renorm(i2, dx2 + d2)
    # axis reflection (Sec. 3.3.3)
    lo, hi = n2 < 0, n2 >= p.n_th
    refl = lo | hi
    n2 = torch.where(lo, torch.zeros_like(n2), torch.where(hi, torch.full_like(n2, p.n_th - 1), n2))
    ndx2 = torch.where(refl, 1.0 - ndx2, ndx2)
    u2 = torch.where(refl, -u[1], u[1])
    leaving = (n1 < 0) | (n1 >= p.n_r)
    out = {
        "i1": torch.where(live, n1, i1), "i2": torch.where(live, n2, i2),
        "dx1": torch.where(live, ndx1, dx1), "dx2": torch.where(live, ndx2, dx2),
        "u1": torch.where(live, u[0], st["u1"]), "u2": torch.where(live, u2, st["u2"]),
        "u3": torch.where(live, u[2], st["u3"]),
        "qm": qm, "m2": m2, "live": live & ~leaving,
    }
    return out


def state_from(P, idx=None):
    """Tensors of a particle dict (numpy SoA as the C oracle holds it)."""
    import numpy as np
    sel = slice(None) if idx is None else idx
    tag = np.asarray(P["tag"][sel])
    sp = tag & 3
    qm = np.where(sp == 1, 1.0, np.where(sp == 2, -1.0, 0.0))
    live = (tag != 0) & ((tag & 0x80) == 0) & ((tag & 0x40) == 0)
    m2 = np.where((tag & 7) == 7, 0.0, 1.0)   # massless neutral: species 3 + bit 0x04
    return {
        "i1": torch.from_numpy(np.asarray(P["i1"][sel], dtype=np.int64)),
        "i2": torch.from_numpy(np.asarray(P["i2"][sel], dtype=np.int64)),
        "dx1": torch.from_numpy(np.asarray(P["dx1"][sel], dtype=np.float64)),
        "dx2": torch.from_numpy(np.asarray(P["dx2"][sel], dtype=np.float64)),
        "u1": torch.from_numpy(np.asarray(P["u1"][sel], dtype=np.float64)),
        "u2": torch.from_numpy(np.asarray(P["u2"][sel], dtype=np.float64)),
        "u3": torch.from_numpy(np.asarray(P["u3"][sel], dtype=np.float64)),
        "qm": torch.from_numpy(qm), "m2": torch.from_numpy(m2), "live": torch.from_numpy(live),
    }


def u_r(p, st):
    """Physical radial covariant component u_r = u_1 / (dr/dx1)."""
    dxi, _ = _grid(p)
    x1 = st["i1"].to(DT) + st["dx1"]
    return st["u1"] / (dxi * (p.r_min - getattr(p, "r0", 0.0)) * torch.exp(x1 * dxi))


def run(p, F1, B0, st, steps):
    for _ in range(steps):
        st = step(p, F1, B0, st)
    return st


def gradients(p, F1, B0, st0, steps):
    """d(mean final u_r)/d(initial u_i) per particle and d/dB0, plus the loss.

    Returns (loss, grad_u (n, 3), grad_B0, final state)."""
    u0 = [st0[k].clone().requires_grad_(True) for k in ("u1", "u2", "u3")]
    b0 = torch.tensor(float(B0), dtype=DT, requires_grad=True)
    st = dict(st0)
    st["u1"], st["u2"], st["u3"] = u0
    fin = run(p, F1, b0, st, steps)
    loss = u_r(p, fin).mean()
    g = torch.autograd.grad(loss, u0 + [b0], allow_unused=True)
    g = [torch.zeros_like(x) if gi is None else gi for gi, x in zip(g, u0 + [b0])]
    return loss.item(), torch.stack(g[:3], 1), g[3].item(), {k: v.detach() for k, v in fin.items()}
