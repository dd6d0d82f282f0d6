"""Python binding of libgrpic.so (include/grpic.h): argument marshalling only.

Every step of the path runs in the HIP library; this module turns torch device
tensors into the C structs and passes the current torch HIP stream.  Importing
it loads libgrpic.so and raises if the library is missing: there is no CPU
fallback.

Storage mirrors the C ABI: a field set is one tensor of shape
(n_planes, n_r + 2 ng, n_th + 2 ng) whose planes are D(3) B(3) D0(3) B0(3) E(3)
H(3) J(3) J0(3) Dinit(3) Binit(3) T(3), plus Dc(3) Bc(3) in the FP32 form
(n_planes = 33 in FP64, 39 in FP32); particles are a dict of 1-D tensors.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_uint64, c_uint8, c_void_p

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgrpic.so")

GRPIC_FP64, GRPIC_FP32 = 0, 1
PRE_PUSH, POST_DEPOSIT = 0, 1
NPLANE = 33
NPLANE_FP32 = 39
PLANES = {"D": 0, "B": 3, "D0": 6, "B0": 9, "E": 12, "H": 15, "J": 18, "J0": 21,
          "Dinit": 24, "Binit": 27, "T": 30, "Dc": 33, "Bc": 36}
TAG_LEAVING = 0x80

PARTICLE_FIELDS = ["i1", "i2", "dx1", "dx2", "u1", "u2", "u3", "w", "phi",
                   "i1p", "i2p", "dx1p", "dx2p", "tag"]
INT_FIELDS = {"i1", "i2", "i1p", "i2p"}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                      "(or python paper_2511_17701_amd/build.py)")
_lib = ctypes.CDLL(LIB_PATH)


class Params(ctypes.Structure):
    _fields_ = [("a", c_double), ("M", c_double), ("r_min", c_double), ("r_max", c_double),
                ("dt", c_double), ("cfl", c_double), ("small_angle", c_double),
                ("charge_scale", c_double), ("iter_tol", c_double), ("n_r", c_int32),
                ("n_th", c_int32),
                ("n_ghost", c_int32), ("n_iter", c_int32), ("n_filter", c_int32),
                ("n_absorb", c_int32), ("precision", c_int32), ("reserved", c_int32),
                ("r0", c_double), ("h0", c_double)]


class Fields(ctypes.Structure):
    _fields_ = [(name, c_void_p * 3) for name in
                ("D", "B", "D0", "B0", "E", "H", "J", "J0", "Dinit", "Binit", "T", "Dc", "Bc")]


class Particles(ctypes.Structure):
    _fields_ = [("n", c_int64), ("i1", c_void_p), ("i2", c_void_p), ("dx1", c_void_p),
                ("dx2", c_void_p), ("u1", c_void_p), ("u2", c_void_p), ("u3", c_void_p),
                ("w", c_void_p), ("phi", c_void_p), ("i1p", c_void_p), ("i2p", c_void_p),
                ("dx1p", c_void_p), ("dx2p", c_void_p), ("tag", c_void_p)]


class InjectParams(ctypes.Structure):
    _fields_ = [("sigma_th", c_double), ("temperature", c_double), ("weight", c_double),
                ("n_pairs", c_int32), ("i_lo", c_int32), ("i_hi", c_int32), ("reserved", c_int32),
                ("seed", c_uint64), ("call", ctypes.c_uint32)]


class Diag(ctypes.Structure):
    _fields_ = [("n_alive", c_int64 * 4), ("n_leaving", c_int64), ("n_empty", c_int64),
                ("n_nonfinite", c_int64), ("sum_E", c_double * 4), ("sum_L", c_double * 4),
                ("gauss_max", c_double), ("gauss_scale", c_double)]


_P, _F, _PP = POINTER(Params), POINTER(Fields), POINTER(Particles)
_sigs = {
    "grpic_last_error": ([], c_char_p),
    "grpic_create": ([_P, POINTER(c_void_p)], c_int32),
    "grpic_destroy": ([c_void_p], c_int32),
    "grpic_get_params": ([c_void_p, _P], c_int32),
    "grpic_particles_init": ([c_void_p, _PP, c_int64, c_int32, c_double, c_int64, c_uint64,
                              c_void_p], c_int32),
    "grpic_fields_init_wald": ([c_void_p, _F, c_double, c_void_p], c_int32),
    "grpic_fields_init_monopole": ([c_void_p, _F, c_double, c_void_p], c_int32),
    "grpic_push": ([c_void_p, _F, _PP, c_void_p], c_int32),
    "grpic_deposit": ([c_void_p, _PP, _F, c_void_p], c_int32),
    "grpic_push_deposit": ([c_void_p, _F, _PP, c_void_p], c_int32),
    "grpic_push_deposit_ranked": ([c_void_p, _F, _PP, c_void_p], c_int32),
    "grpic_push_adjoint": ([c_void_p, _F, c_double, _PP, c_void_p, c_void_p, c_void_p, c_void_p],
                           c_int32),
    "grpic_field_advance": ([c_void_p, _F, c_int32, c_void_p], c_int32),
    "grpic_sort": ([c_void_p, _PP, _PP, POINTER(c_int64), c_void_p], c_int32),
    "grpic_sort_ranked": ([c_void_p, _PP, _PP, POINTER(c_int64), c_void_p], c_int32),
    "grpic_sort_noalloc": ([c_void_p, _PP, _PP, c_void_p, c_void_p], c_int32),
    "grpic_inject_pairs": ([c_void_p, _F, _PP, POINTER(InjectParams), c_int64, POINTER(c_int64),
                            c_void_p], c_int32),
    "grpic_diagnostics": ([c_void_p, _F, _PP, c_double, POINTER(Diag), c_void_p, c_void_p,
                           c_void_p, c_void_p], c_int32),
}
for _name, (_args, _res) in _sigs.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res

EXPORTS = tuple(_sigs)


class GrpicError(RuntimeError):
    pass


def _check(status: int, what: str) -> None:
    if status != 0:
        msg = _lib.grpic_last_error().decode(errors="replace")
        raise GrpicError(f"{what} failed ({status}): {msg}")


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype(precision: int):
    return torch.float64 if precision == GRPIC_FP64 else torch.float32


class Context:
    """A grpic_ctx for the current device.  `params` keys follow grpic_params."""

    def __init__(self, a, M, r_min, r_max, n_r, n_th, dt=0.0, cfl=0.5, n_iter=10,
                 small_angle=1e-5, charge_scale=0.0, n_filter=0, n_absorb=0,
                 precision=GRPIC_FP64, n_ghost=2, iter_tol=0.0, r0=0.0, h0=0.0):
        p = Params(a=a, M=M, r_min=r_min, r_max=r_max, dt=dt, cfl=cfl, small_angle=small_angle,
                   charge_scale=charge_scale, iter_tol=iter_tol, n_r=n_r, n_th=n_th,
                   n_ghost=n_ghost,
                   n_iter=n_iter, n_filter=n_filter, n_absorb=n_absorb, precision=precision,
                   reserved=0, r0=r0, h0=h0)
        h = c_void_p()
        _check(_lib.grpic_create(ctypes.byref(p), ctypes.byref(h)), "grpic_create")
        self._h = h
        q = Params()
        _check(_lib.grpic_get_params(h, ctypes.byref(q)), "grpic_get_params")
        self.params = q
        self.dtype = _dtype(precision)
        self.n_planes = NPLANE_FP32 if precision == GRPIC_FP32 else NPLANE

    @property
    def dt(self) -> float:
        return self.params.dt

    @property
    def shape(self):
        p = self.params
        return (p.n_r + 2 * p.n_ghost, p.n_th + 2 * p.n_ghost)

    def close(self):
        if getattr(self, "_h", None):
            _lib.grpic_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ storage
    def new_fields(self, device="cuda") -> torch.Tensor:
        return torch.zeros((self.n_planes,) + self.shape, dtype=self.dtype, device=device)

    def new_particles(self, n: int, device="cuda") -> dict:
        P = {}
        for k in PARTICLE_FIELDS:
            if k in INT_FIELDS:
                P[k] = torch.zeros(n, dtype=torch.int32, device=device)
            elif k == "tag":
                P[k] = torch.zeros(n, dtype=torch.uint8, device=device)
            else:
                P[k] = torch.zeros(n, dtype=self.dtype, device=device)
        return P

    def _fields(self, F: torch.Tensor) -> Fields:
        if F.shape != (self.n_planes,) + self.shape or F.dtype != self.dtype or \
                not F.is_contiguous():
            raise GrpicError(f"field tensor must be contiguous {self.dtype} of shape "
                             f"{(self.n_planes,) + self.shape}")
        if not F.is_cuda:
            raise GrpicError("field tensor must be on the GPU")
        s = Fields()
        base = F.data_ptr()
        step = F[0].numel() * F.element_size()
        for name, first in PLANES.items():
            if first >= self.n_planes:
                continue
            arr = getattr(s, name)
            for c in range(3):
                arr[c] = base + (first + c) * step
        return s

    def _particles(self, P: dict) -> Particles:
        n = P["tag"].numel()
        s = Particles(n=n)
        for k in PARTICLE_FIELDS:
            t = P[k]
            want = torch.int32 if k in INT_FIELDS else (torch.uint8 if k == "tag" else self.dtype)
            if t.dtype != want or t.numel() != n or not t.is_contiguous() or not t.is_cuda:
                raise GrpicError(f"particle array {k} must be a contiguous GPU {want} of length {n}")
            setattr(s, k, t.data_ptr())
        return s

    # ------------------------------------------------------------ calls
    def particles_init(self, P: dict, n_pairs: int, ppc: int, T: float, n_geo: int, seed: int):
        _check(_lib.grpic_particles_init(self._h, ctypes.byref(self._particles(P)), n_pairs, ppc,
                                         T, n_geo, seed, _stream()), "grpic_particles_init")

    def fields_init_wald(self, F: torch.Tensor, B0: float):
        _check(_lib.grpic_fields_init_wald(self._h, ctypes.byref(self._fields(F)), B0, _stream()),
               "grpic_fields_init_wald")

    def fields_init_monopole(self, F: torch.Tensor, B0: float):
        _check(_lib.grpic_fields_init_monopole(self._h, ctypes.byref(self._fields(F)), B0, _stream()),
               "grpic_fields_init_monopole")

    def push(self, F: torch.Tensor, P: dict):
        _check(_lib.grpic_push(self._h, ctypes.byref(self._fields(F)),
                               ctypes.byref(self._particles(P)), _stream()), "grpic_push")

    def deposit(self, P: dict, F: torch.Tensor):
        _check(_lib.grpic_deposit(self._h, ctypes.byref(self._particles(P)),
                                  ctypes.byref(self._fields(F)), _stream()), "grpic_deposit")

    def push_deposit(self, F: torch.Tensor, P: dict, ranked: bool = False):
        """grpic_push_deposit; ranked: grpic_push_deposit_ranked (the pass
        also ranks the slots for a following sort(P, Q, ranked=True))."""
        if ranked:
            _check(_lib.grpic_push_deposit_ranked(self._h, ctypes.byref(self._fields(F)),
                                                  ctypes.byref(self._particles(P)), _stream()),
                   "grpic_push_deposit_ranked")
            return
        _check(_lib.grpic_push_deposit(self._h, ctypes.byref(self._fields(F)),
                                       ctypes.byref(self._particles(P)), _stream()),
               "grpic_push_deposit")

    def push_adjoint(self, F: torch.Tensor, B0: float, P: dict, gbar_in: torch.Tensor,
                     gbar_out: torch.Tensor, gbar_B0: torch.Tensor):
        """gbar_out = (ds'/ds)^T gbar_in, gbar_B0 += (ds'/dB0) . gbar_in for one
        push step from state P in the frozen field F = B0 F1 (see grpic.h)."""
        n = P["tag"].numel()
        for t, shape in ((gbar_in, (5, n)), (gbar_out, (5, n)), (gbar_B0, (n,))):
            if t.shape != shape or t.dtype != torch.float64 or not t.is_contiguous() or \
                    not t.is_cuda:
                raise GrpicError(f"adjoint arrays must be contiguous GPU float64 of shape {shape}")
        _check(_lib.grpic_push_adjoint(self._h, ctypes.byref(self._fields(F)), B0,
                                       ctypes.byref(self._particles(P)),
                                       c_void_p(gbar_in.data_ptr()), c_void_p(gbar_out.data_ptr()),
                                       c_void_p(gbar_B0.data_ptr()), _stream()),
               "grpic_push_adjoint")

    def field_advance(self, F: torch.Tensor, stage: int):
        _check(_lib.grpic_field_advance(self._h, ctypes.byref(self._fields(F)), stage, _stream()),
               "grpic_field_advance")

    def sort(self, P: dict, Q: dict, count: bool = False, ranked: bool = False):
        """Cell-sort the slots of P into Q (same size); returns the number of
        live slots when count is True (waits for the stream).  ranked:
        grpic_sort_ranked, from the ranks of the preceding
        push_deposit(F, P, ranked=True)."""
        n = c_int64(0)
        fn, name = (_lib.grpic_sort_ranked, "grpic_sort_ranked") if ranked else (_lib.grpic_sort, "grpic_sort")
        _check(fn(self._h, ctypes.byref(self._particles(P)), ctypes.byref(self._particles(Q)),
                  ctypes.byref(n) if count else None, _stream()), name)
        return n.value if count else None

    def sort_noalloc(self, P: dict, Q: dict, n_live=None):
        """grpic_sort_noalloc: the cell sort of P into Q with the library's
        static scratch; n_live: optional int32 device tensor of one element
        that receives the number of live slots (no wait)."""
        if n_live is not None and (n_live.dtype != torch.int32 or not n_live.is_cuda):
            raise ValueError("n_live must be an int32 device tensor")
        _check(_lib.grpic_sort_noalloc(self._h, ctypes.byref(self._particles(P)),
                                       ctypes.byref(self._particles(Q)),
                                       c_void_p(n_live.data_ptr() if n_live is not None else 0),
                                       _stream()), "grpic_sort_noalloc")

    def inject_pairs(self, F: torch.Tensor, P: dict, sigma_th: float, temperature: float,
                     n_pairs: int, weight: float, i_lo: int, i_hi: int, seed: int, call: int,
                     first_free: int, count: bool = True):
        """grpic_inject_pairs: pairs where sigma >= sigma_th into the slots of P
        from first_free on; returns the number written when count is True
        (waits for the stream)."""
        ip = InjectParams(sigma_th=sigma_th, temperature=temperature, weight=weight,
                          n_pairs=n_pairs, i_lo=i_lo, i_hi=i_hi, reserved=0, seed=seed, call=call)
        n = c_int64(0)
        _check(_lib.grpic_inject_pairs(self._h, ctypes.byref(self._fields(F)),
                                       ctypes.byref(self._particles(P)), ctypes.byref(ip),
                                       int(first_free), ctypes.byref(n) if count else None,
                                       _stream()), "grpic_inject_pairs")
        return n.value if count else None

    def diagnostics(self, F: torch.Tensor, P: dict, B0: float, per_particle: bool = False,
                    gauss_plane: bool = False) -> dict:
        n = P["tag"].numel()
        E = torch.empty(n, dtype=self.dtype, device=F.device) if per_particle else None
        L = torch.empty(n, dtype=self.dtype, device=F.device) if per_particle else None
        R = torch.empty(self.shape, dtype=self.dtype, device=F.device) if gauss_plane else None
        d = Diag()
        _check(_lib.grpic_diagnostics(self._h, ctypes.byref(self._fields(F)),
                                      ctypes.byref(self._particles(P)), B0, ctypes.byref(d),
                                      c_void_p(E.data_ptr() if E is not None else 0),
                                      c_void_p(L.data_ptr() if L is not None else 0),
                                      c_void_p(R.data_ptr() if R is not None else 0),
                                      _stream()), "grpic_diagnostics")
        out = {"n_alive": list(d.n_alive), "n_leaving": d.n_leaving, "n_empty": d.n_empty,
               "n_nonfinite": d.n_nonfinite, "sum_E": list(d.sum_E), "sum_L": list(d.sum_L),
               "gauss_max": d.gauss_max, "gauss_scale": d.gauss_scale}
        if per_particle:
            out["E"], out["L"] = E, L
        if gauss_plane:
            out["gauss_res"] = R
        return out

    def step(self, F: torch.Tensor, P: dict, fused: bool = False):
        """One PIC step (Sec. 3.4): pre-push field stage, push, deposit, post-deposit
        stage (push and deposit in one pass when fused)."""
        self.field_advance(F, PRE_PUSH)
        if fused:
            self.push_deposit(F, P)
        else:
            self.push(F, P)
            self.deposit(P, F)
        self.field_advance(F, POST_DEPOSIT)
