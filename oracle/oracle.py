"""ctypes marshalling for liboracle.so (see gc_oracle.h for the meaning of every field)."""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

ACTIVE, EXITED, FINISHED, NONFINITE = 0, 1, 2, 3
BOOTSTRAP, PENDING = 1, 2
FIELD_GRID, FIELD_PARKER, FIELD_CALLBACK = 0, 1, 2
EVAL_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_double, C.c_double, C.c_double, C.POINTER(C.c_double))

PARTICLE_DTYPE = np.dtype([
    ("r", "f8"), ("th", "f8"), ("ph", "f8"), ("u", "f8"), ("mu_B", "f8"),
    ("fp", "f8", (4,)), ("dtp", "f8"), ("s", "f8"), ("ell", "f8"), ("t", "f8"),
    ("k", "u4"), ("flags", "u4"), ("status", "u4"), ("step", "u4"), ("id", "u4"), ("ens", "u4"),
    ("gen", "u4"), ("birth", "u4"),
], align=True)
assert PARTICLE_DTYPE.itemsize == 136


class _Field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nr", C.c_int32), ("nth", C.c_int32), ("nph", C.c_int32),
                ("r_min", C.c_double), ("r_max", C.c_double), ("data", C.c_void_p),
                ("a0", C.c_double), ("omega", C.c_double), ("v_wind", C.c_double),
                ("eval", EVAL_FN), ("user", C.c_void_p), ("extra", C.c_void_p)]


class _Inject(C.Structure):
    _fields_ = [("ekin", C.c_double), ("r0", C.c_double), ("lat0", C.c_double), ("lon0", C.c_double),
                ("dlon", C.c_double), ("dr0", C.c_double), ("dlat", C.c_double),
                ("mu_lo", C.c_double), ("mu_hi", C.c_double)]


class _Ens(C.Structure):
    _fields_ = [("q", C.c_double), ("m", C.c_double), ("lam", C.c_double),
                ("r_in", C.c_double), ("r_out", C.c_double), ("seed", C.c_uint64),
                ("ensemble", C.c_uint32), ("drift_free", C.c_int32), ("max_steps", C.c_int64),
                ("scatter_law", C.c_int32), ("collision_mode", C.c_int32),
                ("rebirth_steps", C.c_int64), ("inj", _Inject), ("v_wind", C.c_double)]


class _Log(C.Structure):
    _fields_ = [("depth", C.c_int32), ("pad", C.c_int32), ("step", C.c_void_p),
                ("mu_new", C.c_void_p), ("ell", C.c_void_p)]


class _MomentSpec(C.Structure):
    _fields_ = [("n_rbins", C.c_int32), ("r_lo", C.c_double), ("r_hi", C.c_double),
                ("n_mubins", C.c_int32), ("sel_r_lo", C.c_double), ("sel_r_hi", C.c_double),
                ("age_lo", C.c_double), ("age_hi", C.c_double), ("min_collisions", C.c_int32),
                ("n_agebins", C.c_int32), ("age_max", C.c_double), ("n_ebins", C.c_int32),
                ("e_lo", C.c_double), ("e_hi", C.c_double), ("e_unit", C.c_double),
                ("len_unit", C.c_double), ("min_birth", C.c_uint32)]


def _load():
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    L = C.CDLL(_LIB_PATH)
    P = C.c_void_p
    L.or_philox4x64_10.argtypes = [P, P, P]
    L.or_u01.argtypes = [C.c_uint64]
    L.or_u01.restype = C.c_double
    L.or_field_eval.argtypes = [C.POINTER(_Field), C.c_double, C.c_double, C.c_double, P]
    L.or_field_eval.restype = C.c_int
    L.or_parker_closed_form.argtypes = [C.c_double] * 5 + [P]
    L.or_rhs.argtypes = [P, C.c_double, C.c_double, C.c_double, C.c_int, P, P, P, P, P]
    L.or_field_eval_extra.argtypes = [C.POINTER(_Field), C.c_double, C.c_double, C.c_double, P]
    L.or_field_eval_extra.restype = C.c_int
    L.or_pc_predict.argtypes = [P, P, P, C.c_double, C.c_double, P]
    L.or_pc_correct.argtypes = [P, P, P, P, C.c_double, C.c_double, P]
    L.or_inject.argtypes = [C.POINTER(_Field), C.POINTER(_Ens), C.c_uint32, P, C.c_int64, P]
    L.or_advance.argtypes = [C.POINTER(_Field), P, P, C.c_int64, C.c_double, C.c_int64, C.c_int, C.POINTER(_Log)]
    L.or_advance_traj.argtypes = [C.POINTER(_Field), P, P, C.c_double, C.c_int64, P]
    L.or_moments_size.argtypes = [C.POINTER(_MomentSpec)]
    L.or_moments_size.restype = C.c_int64
    L.or_moments.argtypes = [C.POINTER(_Field), P, P, C.c_int64, C.POINTER(_MomentSpec), P]
    L.or_max_threads.restype = C.c_int
    return L


lib = _load()


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ----------------------------------------------------------------------------
class Field:
    """A gridded field ([nr][nth][nph][12] float64), the closed-form Parker
    spiral, or a callback fn(r, th, ph) -> 12 components (or None where
    undefined); advance calls with a callback field must use nthreads=1."""

    def __init__(self, grid, data: Optional[np.ndarray] = None, parker: Optional[dict] = None, callback=None,
                 extra: Optional[np.ndarray] = None):
        """extra (grid fields only): [nr][nth][nph][9] node values of (v_E.grad)b,
        (b.grad)v_E and (v_E.grad)v_E; with it the full Eqs. 1-2 are integrated."""
        self.grid = grid
        self.callback = callback
        self.extra = None
        if callback is not None:
            def _eval(_user, r, th, ph, out):
                g = callback(r, th, ph)
                if g is None or not np.all(np.isfinite(g)):
                    return 0
                for c in range(12):
                    out[c] = float(g[c])
                return 1
            self._fn = EVAL_FN(_eval)
            self.data = None
            self._s = _Field(FIELD_CALLBACK, grid.nr, grid.nth, grid.nph, grid.r_min, grid.r_max,
                             None, 0.0, 0.0, 0.0, self._fn, None)
        elif data is not None:
            self.data = np.ascontiguousarray(data, dtype=np.float64)
            assert self.data.shape == (grid.nr, grid.nth, grid.nph, 12)
            self._s = _Field(FIELD_GRID, grid.nr, grid.nth, grid.nph, grid.r_min, grid.r_max,
                             self.data.ctypes.data, 0.0, 0.0, 0.0)
            if extra is not None:
                self.extra = np.ascontiguousarray(extra, dtype=np.float64)
                assert self.extra.shape == (grid.nr, grid.nth, grid.nph, 9)
                self._s.extra = self.extra.ctypes.data
        else:
            self.data = None
            self._s = _Field(FIELD_PARKER, grid.nr, grid.nth, grid.nph, grid.r_min, grid.r_max,
                             None, parker["a0"], parker["omega"], parker["v_wind"])

    @property
    def ref(self):
        return C.byref(self._s)


def philox(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    c = np.array(ctr, dtype=np.uint64)
    k = np.array(key, dtype=np.uint64)
    o = np.zeros(4, dtype=np.uint64)
    lib.or_philox4x64_10(_ptr(c), _ptr(k), _ptr(o))
    return o


def u01(x: int) -> float:
    return lib.or_u01(int(x))


def field_eval(field: Field, r: float, th: float, ph: float):
    o = np.zeros(12)
    ok = lib.or_field_eval(field.ref, r, th, ph, _ptr(o))
    return o, bool(ok)


def parker_closed_form(a0, omega, v, r, th) -> np.ndarray:
    o = np.zeros(12)
    lib.or_parker_closed_form(a0, omega, v, r, th, _ptr(o))
    return o


def field_eval_extra(field: Field, r: float, th: float, ph: float):
    o = np.zeros(9)
    ok = lib.or_field_eval_extra(field.ref, r, th, ph, _ptr(o))
    return o, bool(ok)


def rhs(X, mu_B, q, m, fld, drift_free=False, extra=None):
    """GC right-hand side; extra (9 values) adds the terms of the full Eqs. 1-2."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    fld = np.ascontiguousarray(fld, dtype=np.float64)
    xp = None
    if extra is not None:
        extra = np.ascontiguousarray(extra, dtype=np.float64)
        xp = _ptr(extra)
    F = np.zeros(4)
    vp = C.c_double()
    g = C.c_double()
    lib.or_rhs(_ptr(X), mu_B, q, m, int(drift_free), _ptr(fld), xp, _ptr(F), C.addressof(vp), C.addressof(g))
    return F, vp.value, g.value


def pc_predict(X, Fn, Fp, h, tau):
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (X, Fn, Fp)]
    o = np.zeros(4)
    lib.or_pc_predict(*[_ptr(v) for v in a], h, tau, _ptr(o))
    return o


def pc_correct(X, Fn, Fs, Fp, h, tau):
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (X, Fn, Fs, Fp)]
    o = np.zeros(4)
    lib.or_pc_correct(*[_ptr(v) for v in a], h, tau, _ptr(o))
    return o


def make_ens_table(ensembles, collision_mode: int = 0):
    """ensembles: objects with the attributes of synthetic.workloads.Ensemble."""
    arr = (_Ens * max(1, len(ensembles)))()
    for i, e in enumerate(ensembles):
        inj = _Inject(e.ekin, e.r0, e.lat0, e.lon0, e.dlon, e.dr0, e.dlat, e.mu_lo, e.mu_hi)
        arr[i] = _Ens(e.q, e.m, e.lambda_par, e.r_in, e.r_out, e.seed, e.ensemble, int(e.drift_free),
                      int(e.max_steps), int(e.scatter_law), int(collision_mode),
                      int(getattr(e, "rebirth_steps", 0)), inj, float(getattr(e, "v_wind", 0.0)))
    return arr


def inject(field: Field, ens_table, ens_index: int, ids: np.ndarray) -> np.ndarray:
    """Particles ids of ensemble ens_table[ens_index] (its injection recipe is in the table)."""
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    out = np.zeros(len(ids), dtype=PARTICLE_DTYPE)
    lib.or_inject(field.ref, C.byref(ens_table[ens_index]), ens_index, _ptr(ids), len(ids), _ptr(out))
    return out


def advance(field: Field, ens_table, particles: np.ndarray, dt: float, n_steps: int,
            nthreads: int = 0, log_depth: int = 0):
    """Advance in place.  With log_depth > 0 returns (steps, mu_new, ell) arrays [n][depth]."""
    assert particles.dtype == PARTICLE_DTYPE and particles.flags.c_contiguous
    n = len(particles)
    log = _Log(0, 0, None, None, None)
    logs = None
    if log_depth > 0:
        logs = (np.full((n, log_depth), 0xFFFFFFFF, dtype=np.uint32),
                np.full((n, log_depth), np.nan), np.full((n, log_depth), np.nan))
        log = _Log(log_depth, 0, logs[0].ctypes.data, logs[1].ctypes.data, logs[2].ctypes.data)
    if field.callback is not None:
        nthreads = 1
    lib.or_advance(field.ref, C.cast(ens_table, C.c_void_p), _ptr(particles), n, dt, int(n_steps),
                   int(nthreads), C.byref(log))
    return logs


def advance_traj(field: Field, ens_table, particle: np.ndarray, dt: float, n_steps: int) -> np.ndarray:
    """Advance ONE particle (a length-1 PARTICLE_DTYPE array) recording X after every step."""
    assert particle.dtype == PARTICLE_DTYPE and len(particle) == 1
    traj = np.zeros((n_steps + 1, 4))
    lib.or_advance_traj(field.ref, C.cast(ens_table, C.c_void_p), _ptr(particle), dt, int(n_steps), _ptr(traj))
    return traj


@dataclass
class MomentSpec:
    n_rbins: int = 0
    r_lo: float = 0.0
    r_hi: float = 1.0
    n_mubins: int = 0
    sel_r_lo: float = 0.0
    sel_r_hi: float = 0.0
    age_lo: float = 0.0
    age_hi: float = 0.0
    min_collisions: int = 0
    n_agebins: int = 0
    age_max: float = 1.0
    n_ebins: int = 0
    e_lo: float = 0.0
    e_hi: float = 1.0
    e_unit: float = 1.602176634e-19
    len_unit: float = 1.495978707e11
    min_birth: int = 0

    def _c(self):
        return _MomentSpec(self.n_rbins, self.r_lo, self.r_hi, self.n_mubins, self.sel_r_lo, self.sel_r_hi,
                           self.age_lo, self.age_hi, self.min_collisions, self.n_agebins, self.age_max,
                           self.n_ebins, self.e_lo, self.e_hi, self.e_unit, self.len_unit, self.min_birth)


def moments_size(spec: MomentSpec) -> int:
    s = spec._c()
    return int(lib.or_moments_size(C.byref(s)))


def moments(field: Field, ens_table, particles: np.ndarray, spec: MomentSpec) -> np.ndarray:
    s = spec._c()
    out = np.zeros(moments_size(spec), dtype=np.int64)
    lib.or_moments(field.ref, C.cast(ens_table, C.c_void_p), _ptr(particles), len(particles), C.byref(s), _ptr(out))
    return out


def max_threads() -> int:
    return int(lib.or_max_threads())
