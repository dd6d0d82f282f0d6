"""Synthetic workloads: configuration table and seeded input generators.

This module holds no arithmetic of the method (no metric, tetrad, pusher or
field formula).  It names the configurations of the GRPIC hot path, with their
sizes, and draws plain seeded random arrays (numpy PCG64) for test inputs.  Both
the oracle-side tests and the HIP-side tests and benchmark take their inputs
from here.

Configurations (Kerr, M = 1, log-spaced r from 0.9 r_h, theta in [0, pi], Wald
vacuum field, Maxwell-Juttner pairs, CFL 0.5; deposited charge per unit weight
kappa = 1e-8, a tenuous plasma whose plasma frequency stays far below 1/dt
even in the smallest cells next to the axis, so the Wald field dominates while
every particle still deposits a non-zero current):

========  =====  ======  =========  ====================================  =====  =========
name      a      grid    r_max      particles                             steps  form
========  =====  ======  =========  ====================================  =====  =========
c1_64     0.9    64^2    20         1e5 (5e4 pairs), T = 0.1, B0 = 1      10     FP64
c2_512    0.9    512^2   50         16 ppc + 1e3 neutral geodesics, T=1   100    FP64
c3_2048   0.99   2048^2  100        32 ppc, T = 1, B0 = 10                100    FP32 vs FP64
c4_256    0.9    256^2   20         1e6, T = 1, frozen Wald, B0 learnable 50     adjoint (*)
c5_4096   0.95   4096^2  200        16 ppc (pairs), T = 1, B0 = 10        200    FP32 full step
c6_mono   0.2    2048^2  10         90 ppc (pairs), T = 0.5, B0 = 1       100    FP64 full step
c7_qks    0.2    2048^2  10         as c6, quasi-spherical r0 = 0.5, h0=0.3 100   FP64 full step
========  =====  ======  =========  ====================================  =====  =========

c6_monopole is the paper's own benchmark shape: the BZ monopole test
(A_phi = -B0 cos theta, D = 0) on a 2048^2 log-r x theta mesh with 90 particles
per cell, r from r_g to 10 r_g with an absorbing layer 1 r_g thick (94 cells),
pairs at the test's injection temperature T = 0.5.  c7_qks_monopole is the same
shape on the general quasi-spherical map of App. A (xi = log(r - 0.5), points
concentrated toward the equator with h0 = 0.3).

(*) the differentiation form runs the implicit iterations to their fixed
points (up to 200 iterations, stopping at an exact repeat), as its
implicit-function-theorem adjoint assumes: a passage within ~1e-3 rad of the
axis contracts by only ~0.8 per iteration.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    a: float
    n_r: int
    n_th: int
    r_max: float
    B0: float
    T: float
    n_pairs: int          # used when ppc == 0
    ppc: int              # particles per cell (pairs: ppc/2 per cell)
    n_geo: int            # neutral test geodesics
    steps: int
    precision: str        # "fp64" | "fp32"
    n_filter: int = 0
    n_absorb: int = 0
    M: float = 1.0
    cfl: float = 0.5
    n_iter: int = 10
    small_angle: float = 1e-5
    seed: int = 0
    charge_scale: float = 1e-8
    ng: int = 2
    full_step: bool = False    # field_advance inside the step
    init: str = "wald"         # initial field: "wald" | "monopole"
    r_inner: float = 0.0       # inner radius (0: 0.9 r_h)
    r0: float = 0.0            # quasi-spherical map (App. A): xi = log(r - r0)
    h0: float = 0.0            # and equatorial concentration of theta(eta)

    @property
    def r_h(self) -> float:
        return self.M + math.sqrt(self.M * self.M - self.a * self.a)

    @property
    def r_min(self) -> float:
        return self.r_inner if self.r_inner > 0 else 0.9 * self.r_h

    @property
    def n_particles(self) -> int:
        if self.ppc > 0:
            return self.n_r * self.n_th * self.ppc + self.n_geo
        return 2 * self.n_pairs + self.n_geo

    @property
    def n_pairs_total(self) -> int:
        if self.ppc > 0:
            return self.n_r * self.n_th * self.ppc // 2
        return self.n_pairs

    def scaled(self, n_r: int, n_th: int, **kw) -> "Workload":
        """Same physics on a smaller grid (for oracle-sized parity cases)."""
        return replace(self, n_r=n_r, n_th=n_th, **kw)


WORKLOADS = {
    "c1_64": Workload("c1_64", a=0.9, n_r=64, n_th=64, r_max=20.0, B0=1.0, T=0.1,
                      n_pairs=50_000, ppc=0, n_geo=0, steps=10, precision="fp64"),
    "c2_512": Workload("c2_512", a=0.9, n_r=512, n_th=512, r_max=50.0, B0=1.0, T=1.0,
                       n_pairs=0, ppc=16, n_geo=1000, steps=100, precision="fp64",
                       full_step=True),
    "c3_2048": Workload("c3_2048", a=0.99, n_r=2048, n_th=2048, r_max=100.0, B0=10.0, T=1.0,
                        n_pairs=0, ppc=32, n_geo=0, steps=100, precision="fp32",
                        full_step=True),
    "c4_256": Workload("c4_256", a=0.9, n_r=256, n_th=256, r_max=20.0, B0=1.0, T=1.0,
                       n_pairs=500_000, ppc=0, n_geo=0, steps=50, precision="fp64",
                       n_iter=200),
    "c5_4096": Workload("c5_4096", a=0.95, n_r=4096, n_th=4096, r_max=200.0, B0=10.0, T=1.0,
                        n_pairs=0, ppc=16, n_geo=0, steps=200, precision="fp32",
                        n_filter=4, n_absorb=32, full_step=True),
    "c6_monopole": Workload("c6_monopole", a=0.2, n_r=2048, n_th=2048, r_max=10.0, B0=1.0, T=0.5,
                            n_pairs=0, ppc=90, n_geo=0, steps=100, precision="fp64",
                            n_absorb=94, full_step=True, init="monopole", r_inner=1.0),
    "c7_qks_monopole": Workload("c7_qks_monopole", a=0.2, n_r=2048, n_th=2048, r_max=10.0,
                                B0=1.0, T=0.5, n_pairs=0, ppc=90, n_geo=0, steps=100,
                                precision="fp64", n_absorb=94, full_step=True, init="monopole",
                                r_inner=1.0, r0=0.5, h0=0.3),
}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_positions(n: int, n_r: int, n_th: int, seed: int, i1_range=None, i2_range=None):
    """Uniform cell indices and in-cell offsets (int32 cell, float64 offset in [0, 1))."""
    g = rng(seed)
    lo1, hi1 = i1_range if i1_range else (0, n_r)
    lo2, hi2 = i2_range if i2_range else (0, n_th)
    i1 = g.integers(lo1, hi1, size=n, dtype=np.int32)
    i2 = g.integers(lo2, hi2, size=n, dtype=np.int32)
    dx1 = g.random(n)
    dx2 = g.random(n)
    return i1, dx1, i2, dx2


def random_normal(n: int, scale: float, seed: int) -> np.ndarray:
    return rng(seed).normal(0.0, scale, size=n)


def random_uniform(shape, lo: float, hi: float, seed: int) -> np.ndarray:
    return rng(seed).uniform(lo, hi, size=shape)
