"""Small helpers shared by the tests: placing single particles at physical
positions and converting physical (r, theta, phi) components to code units.

Code coordinates (App. A, quasi-spherical map with r0 = h0 = 0):
x1 = ln(r / r_min) / dxi, x2 = theta / dth, covariant u_1 = u_r * dxi * r,
u_2 = u_theta * dth, u_3 = u_phi.
"""
import math

import numpy as np


def grid(r_min, r_max, n_r, n_th):
    return math.log(r_max / r_min) / n_r, math.pi / n_th


def place(P, k, r, th, r_min, dxi, dth):
    x1 = math.log(r / r_min) / dxi
    x2 = th / dth
    P["i1"][k] = int(math.floor(x1)); P["dx1"][k] = x1 - math.floor(x1)
    P["i2"][k] = int(math.floor(x2)); P["dx2"][k] = x2 - math.floor(x2)
    for c in ("i1", "dx1", "i2", "dx2"):
        P[c + "p"][k] = P[c][k]


def position(P, k, r_min, dxi, dth, prev=False):
    s = "p" if prev else ""
    x1 = P["i1" + s][k] + P["dx1" + s][k]
    x2 = P["i2" + s][k] + P["dx2" + s][k]
    return r_min * math.exp(x1 * dxi), x2 * dth


def single(O, prm, r, th, u_r, u_th, u_phi, tag, w=1.0):
    dxi, dth = grid(prm.r_min, prm.r_max, prm.n_r, prm.n_th)
    P = O.new_particles(1)
    place(P, 0, r, th, prm.r_min, dxi, dth)
    P["u1"][0] = u_r * dxi * r
    P["u2"][0] = u_th * dth
    P["u3"][0] = u_phi
    P["w"][0] = w
    P["tag"][0] = tag
    return P


def cartesian(r, th, ph):
    return np.array([r * math.sin(th) * math.cos(ph), r * math.sin(th) * math.sin(ph),
                     r * math.cos(th)])


def bl_energy(a, M, r, th, L):
    """Energy of a particle with Boyer-Lindquist u_r = u_theta = 0 and angular
    momentum L (textbook BL Kerr metric), and its Kerr-Schild u_r from the
    transformation of Sec. 4.1 (eq. BL-KS-transformation)."""
    Sig = r * r + a * a * math.cos(th) ** 2
    Del = r * r - 2 * M * r + a * a
    s2 = math.sin(th) ** 2
    gtt = -(1 - 2 * M * r / Sig)
    gtp = -2 * M * a * r * s2 / Sig
    gpp = (r * r + a * a + 2 * M * a * a * r * s2 / Sig) * s2
    det = gtt * gpp - gtp * gtp
    Gtt, Gtp, Gpp = gpp / det, -gtp / det, gtt / det
    A, B, C = Gtt, -2 * Gtp * L, Gpp * L * L + 1
    disc = math.sqrt(B * B - 4 * A * C)
    E = max((-B + disc) / (2 * A), (-B - disc) / (2 * A))
    u_r = -(2 * M * r * (-E) + a * L) / Del
    return E, u_r


def fit_circle(x, y):
    """Algebraic least-squares circle fit; returns centre and radius."""
    A = np.column_stack([x, y, np.ones_like(x)])
    b = x * x + y * y
    c = np.linalg.lstsq(A, b, rcond=None)[0]
    cx, cy = c[0] / 2, c[1] / 2
    return cx, cy, math.sqrt(c[2] + cx * cx + cy * cy)
