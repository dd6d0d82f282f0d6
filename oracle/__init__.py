"""Plain FP64 CPU oracle of the GRPIC hot path (ctypes wrapper over grpic_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py, never by the product path.  It shares no code with
the HIP library; both use the same plain array layouts:

* a field set is an array of shape (33, n_r + 2 ng, n_th + 2 ng) float64 whose
  planes are, in order, D(3) B(3) D0(3) B0(3) E(3) H(3) J(3) J0(3) Dinit(3)
  Binit(3) T(3): em, em0, aux, cur, cur0, absorbing targets, scratch
  (Sec. 3.3, Sec. 3.4 storage of the paper);
* particles are a dict of 1-D arrays i1 i2 (int32), dx1 dx2 u1 u2 u3 w phi
  (float64), i1p i2p (int32), dx1p dx2p (float64), tag (uint8).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from ctypes import POINTER, c_double, c_int, c_int32, c_int64, c_uint8, c_uint32, c_uint64

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "grpic_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

NPLANE = 33
PLANES = {"D": 0, "B": 3, "D0": 6, "B0": 9, "E": 12, "H": 15, "J": 18, "J0": 21,
          "Dinit": 24, "Binit": 27, "T": 30}
TAG_LEAVING = 0x80

PARTICLE_FIELDS = [("i1", np.int32), ("i2", np.int32), ("dx1", np.float64), ("dx2", np.float64),
                   ("u1", np.float64), ("u2", np.float64), ("u3", np.float64), ("w", np.float64),
                   ("phi", np.float64), ("i1p", np.int32), ("i2p", np.int32),
                   ("dx1p", np.float64), ("dx2p", np.float64), ("tag", np.uint8)]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                        "-Wall", "-Wno-unused-function", "-o", tmp, SRC, "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


class Params(ctypes.Structure):
    _fields_ = [("a", c_double), ("M", c_double), ("r_min", c_double), ("r_max", c_double),
                ("dt", c_double), ("small_angle", c_double), ("charge_scale", c_double),
                ("n_r", c_int32), ("n_th", c_int32), ("ng", c_int32), ("n_iter", c_int32),
                ("n_filter", c_int32), ("n_absorb", c_int32), ("r0", c_double), ("h0", c_double)]

    @classmethod
    def make(cls, a, M, r_min, r_max, n_r, n_th, dt, n_iter=10, ng=2, small_angle=1e-5,
             charge_scale=0.0, n_filter=0, n_absorb=0, r0=0.0, h0=0.0):
        """r0, h0: the quasi-spherical map (App. A), xi = log(r - r0) and the
        equatorial concentration h0 of theta(eta); 0, 0 is log r, uniform theta."""
        return cls(a=a, M=M, r_min=r_min, r_max=r_max, dt=dt, small_angle=small_angle,
                   charge_scale=charge_scale, n_r=n_r, n_th=n_th, ng=ng, n_iter=n_iter,
                   n_filter=n_filter, n_absorb=n_absorb, r0=r0, h0=h0)

    def shape(self):
        return (self.n_r + 2 * self.ng, self.n_th + 2 * self.ng)


class Particles(ctypes.Structure):
    _fields_ = [("n", c_int64), ("i1", POINTER(c_int32)), ("i2", POINTER(c_int32)),
                ("dx1", POINTER(c_double)), ("dx2", POINTER(c_double)),
                ("u1", POINTER(c_double)), ("u2", POINTER(c_double)), ("u3", POINTER(c_double)),
                ("w", POINTER(c_double)), ("phi", POINTER(c_double)),
                ("i1p", POINTER(c_int32)), ("i2p", POINTER(c_int32)),
                ("dx1p", POINTER(c_double)), ("dx2p", POINTER(c_double)),
                ("tag", POINTER(c_uint8))]


_MET = ["r", "th", "s", "c", "R", "T", "dT", "Sig", "Del", "A", "S2", "alpha", "beta1",
        "hu11", "hu22", "hu33", "hu13", "hl11", "hl22", "hl33", "hl13", "sqrt_h", "sqrt_ht"]
_DER = ["d_alpha", "d_beta1", "d_hu11", "d_hu22", "d_hu33", "d_hu13"]


class Metric(ctypes.Structure):
    _fields_ = [(k, c_double) for k in _MET] + [(k, c_double * 2) for k in _DER]

    def as_dict(self):
        d = {k: getattr(self, k) for k in _MET}
        for k in _DER:
            v = getattr(self, k)
            d[k] = (v[0], v[1])
        return d


_lib = None


def _load(path):
    L = ctypes.CDLL(path)
    P, PP, D = POINTER(Params), POINTER(Particles), POINTER(c_double)
    L.orc_plane_size.argtypes = [P]; L.orc_plane_size.restype = c_int64
    L.orc_metric_at.argtypes = [P, c_double, c_double, c_int, POINTER(Metric)]
    for nm in ("orc_cov_to_hat", "orc_hat_to_cov", "orc_con_to_hat", "orc_hat_to_con"):
        getattr(L, nm).argtypes = [POINTER(Metric), D, D]
    L.orc_boris.argtypes = [D, D, D, c_double, c_double]
    L.orc_push.argtypes = [P, D, PP]
    L.orc_deposit.argtypes = [P, D, PP]
    L.orc_charge.argtypes = [P, PP, D]
    L.orc_wald_potential.argtypes = [P, c_double, c_double, c_double, D]
    L.orc_wald_fields.argtypes = [P, c_double, c_double, c_double, D, D]
    L.orc_field_advance.argtypes = [P, D, c_int]
    L.orc_fields_init_wald.argtypes = [P, D, c_double]
    L.orc_fields_init_monopole.argtypes = [P, D, c_double]
    L.orc_philox4x32_10.argtypes = [POINTER(c_uint32), POINTER(c_uint32), POINTER(c_uint32)]
    L.orc_particles_init.argtypes = [P, PP, c_int64, c_int32, c_double, c_int64, c_uint64]
    L.orc_energy_momentum.argtypes = [P, PP, c_double, D, D]
    L.orc_gauss_residual.argtypes = [P, D, PP, D, D, D]
    L.orc_gauss_residual.restype = c_double
    L.orc_courant_dt.argtypes = [P, c_double]
    L.orc_courant_dt.restype = c_double
    L.orc_num_threads.restype = c_int
    L.orc_set_num_threads.argtypes = [c_int]
    L.orc_inject_pairs.argtypes = [P, D, PP, c_double, c_double, c_int32, c_double, c_int32,
                                   c_int32, c_uint64, c_uint32, c_int64]
    L.orc_inject_pairs.restype = c_int64
    L.orc_magnetisation.argtypes = [P, D, PP, D]
    L.orc_wald_potential_planes.argtypes = [P, c_double, D, D]
    L.orc_sqrt_h_plane.argtypes = [P, c_int, c_int, D]
    L.orc_gather.argtypes = [P, D, c_int32, c_double, c_int32, c_double, D, D]
    L.orc_axis_bc.argtypes = [P, D, c_int]
    L.orc_field_bc.argtypes = [P, D, D, c_int]
    L.orc_filter_currents.argtypes = [P, D]
    L.orc_match_lambda.argtypes = [P, c_double]
    L.orc_match_lambda.restype = c_double
    return L


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = _load(LIB)
    return _lib


class planted:
    """Context manager for planted-mistake checks of the pins: compiles a copy
    of grpic_oracle.c with each (old, new) text replacement applied (each `old`
    must occur exactly once) into a temporary library and routes every oracle
    call through it until the context ends."""

    def __init__(self, *patches):
        self.patches = patches

    def __enter__(self):
        import tempfile
        src = open(SRC).read()
        for old, new in self.patches:
            assert src.count(old) == 1, "planted mistake: text to replace not found once: %r" % old
            src = src.replace(old, new)
        self._dir = tempfile.TemporaryDirectory()
        c = os.path.join(self._dir.name, "planted.c")
        so = os.path.join(self._dir.name, "libplanted.so")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-w", "-o", so, c,
                        "-lm"], check=True)
        global _lib
        self._saved = lib()
        _lib = _load(so)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self._saved
        self._dir.cleanup()
        return False


def _dp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(POINTER(c_double))


def _pstruct(P):
    n = len(P["tag"])
    s = Particles(n=n)
    for k, dt in PARTICLE_FIELDS:
        arr = P[k]
        assert arr.dtype == dt and arr.flags.c_contiguous and len(arr) == n, k
        ct = {np.int32: c_int32, np.float64: c_double, np.uint8: c_uint8}[dt]
        setattr(s, k, arr.ctypes.data_as(POINTER(ct)))
    return s


# ------------------------------------------------------------------- API

def metric_at(prm: Params, x1: float, x2: float, clamp: bool = True) -> dict:
    m = Metric()
    lib().orc_metric_at(ctypes.byref(prm), x1, x2, int(clamp), ctypes.byref(m))
    return m.as_dict()


def _metric_struct(prm, x1, x2, clamp=True):
    m = Metric()
    lib().orc_metric_at(ctypes.byref(prm), x1, x2, int(clamp), ctypes.byref(m))
    return m


def tetrad(prm: Params, x1: float, x2: float, kind: str, vec, clamp: bool = True):
    """kind in cov_to_hat, hat_to_cov, con_to_hat, hat_to_con."""
    m = _metric_struct(prm, x1, x2, clamp)
    a = np.ascontiguousarray(vec, dtype=np.float64)
    out = np.zeros(3)
    getattr(lib(), "orc_" + kind)(ctypes.byref(m), _dp(a), _dp(out))
    return out


def boris(u, E, B, qm, tau):
    u = np.array(u, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    lib().orc_boris(_dp(u), _dp(E), _dp(B), qm, tau)
    return u


def philox4x32_10(ctr, key):
    c = (c_uint32 * 4)(*ctr)
    k = (c_uint32 * 2)(*key)
    o = (c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def new_fields(prm: Params) -> np.ndarray:
    return np.zeros((NPLANE,) + prm.shape(), dtype=np.float64)


def new_particles(n: int) -> dict:
    return {k: np.zeros(n, dtype=dt) for k, dt in PARTICLE_FIELDS}


def fields_init_wald(prm: Params, B0: float) -> np.ndarray:
    F = new_fields(prm)
    lib().orc_fields_init_wald(ctypes.byref(prm), _dp(F), B0)
    return F


def fields_init_monopole(prm: Params, B0: float) -> np.ndarray:
    """Monopole initial data of the BZ test: A_phi = -B0 cos(theta), D = 0."""
    F = new_fields(prm)
    lib().orc_fields_init_monopole(ctypes.byref(prm), _dp(F), B0)
    return F


def particles_init(prm: Params, n_pairs: int, ppc: int, T: float, n_geo: int, seed: int) -> dict:
    if ppc > 0:
        assert ppc % 2 == 0
        n_pairs = prm.n_r * prm.n_th * ppc // 2
    P = new_particles(2 * n_pairs + n_geo)
    s = _pstruct(P)
    lib().orc_particles_init(ctypes.byref(prm), ctypes.byref(s), n_pairs, ppc, T, n_geo, seed)
    return P


def push(prm: Params, F: np.ndarray, P: dict) -> None:
    s = _pstruct(P)
    lib().orc_push(ctypes.byref(prm), _dp(F), ctypes.byref(s))


def deposit(prm: Params, F: np.ndarray, P: dict) -> None:
    s = _pstruct(P)
    lib().orc_deposit(ctypes.byref(prm), _dp(F), ctypes.byref(s))


def charge(prm: Params, P: dict) -> np.ndarray:
    out = np.zeros(prm.shape())
    s = _pstruct(P)
    lib().orc_charge(ctypes.byref(prm), ctypes.byref(s), _dp(out))
    return out


def field_advance(prm: Params, F: np.ndarray, stage: int) -> None:
    lib().orc_field_advance(ctypes.byref(prm), _dp(F), int(stage))


# parts of the step, called on their own by the pins

def gather(prm: Params, F: np.ndarray, x1: float, x2: float):
    """(D, B) interpolated at code position (x1, x2) from planes D and B0."""
    i1, i2 = int(np.floor(x1)), int(np.floor(x2))
    D, B = np.zeros(3), np.zeros(3)
    lib().orc_gather(ctypes.byref(prm), _dp(F), i1, x1 - i1, i2, x2 - i2, _dp(D), _dp(B))
    return D, B


def axis_bc(prm: Params, X: np.ndarray, kind: int) -> None:
    """Axis ghosts of a triple X (3 planes): kind 0 D-like, 1 B-like, 2 current."""
    lib().orc_axis_bc(ctypes.byref(prm), _dp(X), int(kind))


def field_bc(prm: Params, X: np.ndarray, Xinit: np.ndarray, kind: int) -> None:
    lib().orc_field_bc(ctypes.byref(prm), _dp(X), _dp(Xinit), int(kind))


def filter_currents(prm: Params, F: np.ndarray) -> None:
    lib().orc_filter_currents(ctypes.byref(prm), _dp(F))


def match_lambda(prm: Params, x: float) -> float:
    return lib().orc_match_lambda(ctypes.byref(prm), float(x))


def wald_potential(prm: Params, x1: float, x2: float, B0: float):
    out = np.zeros(3)
    lib().orc_wald_potential(ctypes.byref(prm), x1, x2, B0, _dp(out))
    return out


def wald_fields(prm: Params, x1: float, x2: float, B0: float):
    D = np.zeros(3)
    B = np.zeros(3)
    lib().orc_wald_fields(ctypes.byref(prm), x1, x2, B0, _dp(D), _dp(B))
    return D, B


def inject_pairs(prm: Params, F: np.ndarray, P: dict, sigma_th: float, T: float, n_inj: int,
                 w_inj: float, i_lo: int, i_hi: int, seed: int, call: int, first_free: int) -> int:
    """Pair injection where sigma >= sigma_th (Sec. 4.4, 4.5; reading R30): writes the
    new pairs into slots first_free, first_free + 1, ... of P and returns their count."""
    s = _pstruct(P)
    return lib().orc_inject_pairs(ctypes.byref(prm), _dp(F), ctypes.byref(s), sigma_th, T,
                                  int(n_inj), w_inj, int(i_lo), int(i_hi), int(seed), int(call),
                                  int(first_free))


def magnetisation(prm: Params, F: np.ndarray, P: dict) -> np.ndarray:
    """sigma = B_i B^i / (4 pi n) at every cell centre, shape (n_r, n_th)."""
    out = np.zeros((prm.n_r, prm.n_th))
    s = _pstruct(P)
    lib().orc_magnetisation(ctypes.byref(prm), _dp(F), ctypes.byref(s), _dp(out))
    return out


def energy_momentum(prm: Params, P: dict, B0: float):
    n = len(P["tag"])
    E = np.zeros(n)
    L = np.zeros(n)
    s = _pstruct(P)
    lib().orc_energy_momentum(ctypes.byref(prm), ctypes.byref(s), B0, _dp(E), _dp(L))
    return E, L


def gauss_residual(prm: Params, F: np.ndarray, P: dict):
    res = np.zeros(prm.shape())
    tmp = np.zeros(prm.shape())
    scale = c_double(0.0)
    s = _pstruct(P)
    mx = lib().orc_gauss_residual(ctypes.byref(prm), _dp(F), ctypes.byref(s), _dp(res),
                                  _dp(tmp), ctypes.byref(scale))
    return res, mx, scale.value


def wald_potential_planes(prm: Params, B0: float):
    """(A_1 at r-edges, A_3 at nodes) as planes; test error bounds only."""
    A1 = np.zeros(prm.shape())
    A3 = np.zeros(prm.shape())
    lib().orc_wald_potential_planes(ctypes.byref(prm), B0, _dp(A1), _dp(A3))
    return A1, A3


def sqrt_h_plane(prm: Params, o1: int, o2: int) -> np.ndarray:
    out = np.zeros(prm.shape())
    lib().orc_sqrt_h_plane(ctypes.byref(prm), o1, o2, _dp(out))
    return out


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    """OpenMP thread count of later oracle calls (for timing the oracle)."""
    lib().orc_set_num_threads(int(n))


def courant_dt(prm: Params, cfl: float) -> float:
    return lib().orc_courant_dt(ctypes.byref(prm), cfl)


def step(prm: Params, F: np.ndarray, P: dict) -> None:
    """One PIC step of Sec. 3.4: pre-push field stage, push, deposit, post-deposit stage."""
    field_advance(prm, F, 0)
    push(prm, F, P)
    deposit(prm, F, P)
    field_advance(prm, F, 1)
