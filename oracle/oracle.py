"""ctypes marshalling for the FP64 oracle in ``hlbm_oracle.c``.

Test infrastructure only (see the package docstring).  Arrays are numpy float64
in the oracle's own population ordering, ``g[i, cell]`` with
``cell = x + nx*(y + ny*z)``; :func:`lattice` returns that ordering.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

PERIODIC, WALL, INLET_U, OUTLET_RHO = 0, 1, 2, 3

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hlbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile ``hlbm_oracle.c`` into ``liboracle.so`` (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11", "-Wall",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("q", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("tau", ctypes.c_double),
        ("force", ctypes.c_double * 3),
        ("bc_lo", ctypes.c_int * 3),
        ("bc_hi", ctypes.c_int * 3),
        ("inlet_u", ctypes.c_double * 3),
        ("outlet_rho", ctypes.c_double),
        ("rho0", ctypes.c_double),
    ]


@dataclass
class OracleConfig:
    q: int
    nx: int
    ny: int
    nz: int = 1
    tau: float = 0.6
    force: tuple = (0.0, 0.0, 0.0)
    bc_lo: tuple = (PERIODIC, PERIODIC, PERIODIC)
    bc_hi: tuple = (PERIODIC, PERIODIC, PERIODIC)
    inlet_u: tuple = (0.0, 0.0, 0.0)
    outlet_rho: float = 1.0
    rho0: float = 1.0
    extra: dict = field(default_factory=dict)

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    def c_struct(self) -> _Cfg:
        s = _Cfg()
        s.q, s.nx, s.ny, s.nz = self.q, self.nx, self.ny, self.nz
        s.tau = self.tau
        s.force = (ctypes.c_double * 3)(*self.force)
        s.bc_lo = (ctypes.c_int * 3)(*self.bc_lo)
        s.bc_hi = (ctypes.c_int * 3)(*self.bc_hi)
        s.inlet_u = (ctypes.c_double * 3)(*self.inlet_u)
        s.outlet_rho = self.outlet_rho
        s.rho0 = self.rho0
        return s

    def solid_mask(self) -> np.ndarray:
        """Boolean mask of wall-layer cells, shape (nz, ny, nx)."""
        m = np.zeros((self.nz, self.ny, self.nx), dtype=bool)
        n = (self.nx, self.ny, self.nz)
        for a in range(3):
            ax = 2 - a  # numpy axis of lattice axis a
            if self.bc_lo[a] == WALL:
                sl = [slice(None)] * 3
                sl[ax] = 0
                m[tuple(sl)] = True
            if self.bc_hi[a] == WALL:
                sl = [slice(None)] * 3
                sl[ax] = n[a] - 1
                m[tuple(sl)] = True
        return m


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        D = P(ctypes.c_double)
        C = P(_Cfg)
        lib.oracle_lattice.argtypes = [ctypes.c_int, P(ctypes.c_int), D]
        lib.oracle_equilibrium.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, D, D]
        lib.oracle_equilibrium.restype = None
        lib.oracle_collide_cell.argtypes = [C, ctypes.c_double, D, D]
        lib.oracle_stream.argtypes = [C, D, D, ctypes.c_int]
        lib.oracle_collide.argtypes = [C, D, D, D, ctypes.c_int]
        lib.oracle_moments.argtypes = [C, D, D, D]
        lib.oracle_run.argtypes = [C, D, ctypes.c_int, D, ctypes.c_int]
        lib.oracle_observe.argtypes = [C, D, D, D, ctypes.c_int]
        lib.oracle_max_threads.argtypes = []
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (rc={rc})")


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def lattice(q: int):
    """Return (c[q,3] int, w[q] float64) in the oracle's ordering."""
    c = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q, dtype=np.float64)
    _check(_load().oracle_lattice(q, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w)),
           "lattice")
    return c.astype(np.int64), w


def equilibrium(q: int, rho: float, u, rho0: float = 1.0) -> np.ndarray:
    uu = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(3))
    geq = np.zeros(q, dtype=np.float64)
    _load().oracle_equilibrium(q, rho0, rho, _dp(uu), _dp(geq))
    return geq


def collide_cell(cfg: OracleConfig, d: float, gpre) -> np.ndarray:
    gin = np.ascontiguousarray(np.asarray(gpre, dtype=np.float64))
    gout = np.zeros(cfg.q, dtype=np.float64)
    s = cfg.c_struct()
    _check(_load().oracle_collide_cell(ctypes.byref(s), float(d), _dp(gin), _dp(gout)),
           "collide_cell")
    return gout


def _state(cfg: OracleConfig, g):
    if g is None:
        return np.zeros((cfg.q, cfg.ncells), dtype=np.float64)
    g = np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(cfg.q, cfg.ncells))
    return g.copy()


def _field(cfg: OracleConfig, d):
    d = np.ascontiguousarray(np.asarray(d, dtype=np.float64).reshape(cfg.ncells))
    return d


def stream(cfg: OracleConfig, post, nthreads: int = 1) -> np.ndarray:
    post = _state(cfg, post)
    pre = np.zeros_like(post)
    s = cfg.c_struct()
    _check(_load().oracle_stream(ctypes.byref(s), _dp(post), _dp(pre), nthreads), "stream")
    return pre


def collide(cfg: OracleConfig, d, pre, nthreads: int = 1) -> np.ndarray:
    pre = _state(cfg, pre)
    post = np.zeros_like(pre)
    dd = _field(cfg, d)
    s = cfg.c_struct()
    _check(_load().oracle_collide(ctypes.byref(s), _dp(dd), _dp(pre), _dp(post), nthreads),
           "collide")
    return post


def moments(cfg: OracleConfig, pre):
    """Moments of pre-collision populations -> (drho[N], u[3, N])."""
    pre = _state(cfg, pre)
    drho = np.zeros(cfg.ncells)
    u = np.zeros((3, cfg.ncells))
    s = cfg.c_struct()
    _check(_load().oracle_moments(ctypes.byref(s), _dp(pre), _dp(drho), _dp(u)), "moments")
    return drho, u


def run(cfg: OracleConfig, d, nsteps: int, g=None, nthreads: int = 1) -> np.ndarray:
    """Advance the post-collision state ``g`` (default: rest) by ``nsteps``."""
    g = _state(cfg, g)
    dd = _field(cfg, d)
    s = cfg.c_struct()
    _check(_load().oracle_run(ctypes.byref(s), _dp(dd), int(nsteps), _dp(g), nthreads), "run")
    return g


def observe(cfg: OracleConfig, g, nthreads: int = 1):
    """Moments (drho[N], u[3, N]) at the time level of post-collision state ``g``."""
    g = _state(cfg, g)
    drho = np.zeros(cfg.ncells)
    u = np.zeros((3, cfg.ncells))
    s = cfg.c_struct()
    _check(_load().oracle_observe(ctypes.byref(s), _dp(g), _dp(drho), _dp(u), nthreads),
           "observe")
    return drho, u


# ---------------------------------------------------------------------------
# Discrete adjoint
# ---------------------------------------------------------------------------
def _adj_load():
    lib = _load()
    if not getattr(lib, "_adj_ready", False):
        P = ctypes.POINTER
        D = P(ctypes.c_double)
        C = P(_Cfg)
        lib.oracle_collide_adjoint.argtypes = [C, D, D, D, D, D, ctypes.c_int]
        lib.oracle_stream_adjoint.argtypes = [C, D, D, D]
        lib.oracle_moments_adjoint.argtypes = [C, D, D, D, D]
        lib.oracle_gradient.argtypes = [C, D, ctypes.c_int, ctypes.c_int, D, D, D, ctypes.c_int]
        lib._adj_ready = True
    return lib


def _tensor_load():
    lib = _load()
    if not getattr(lib, "_tensor_ready", False):
        P = ctypes.POINTER
        D = P(ctypes.c_double)
        C = P(_Cfg)
        lib.oracle_collide_cell_tensor.argtypes = [C, D, D, D]
        lib.oracle_collide_tensor.argtypes = [C, D, D, D, ctypes.c_int]
        lib.oracle_run_tensor.argtypes = [C, D, ctypes.c_int, D, ctypes.c_int]
        lib.oracle_collide_adjoint_tensor.argtypes = [C, D, D, D, D, D, ctypes.c_int]
        lib.oracle_gradient_tensor.argtypes = [C, D, ctypes.c_int, ctypes.c_int, D, D, D, ctypes.c_int]
        lib._tensor_ready = True
    return lib


def _tensor_field(cfg: OracleConfig, D6):
    return np.ascontiguousarray(np.asarray(D6, dtype=np.float64).reshape(6, cfg.ncells))


def collide_cell_tensor(cfg: OracleConfig, D6, gpre) -> np.ndarray:
    """One cell with u_eq = (I - D) u; D6 = (xx, yy, zz, xy, xz, yz)."""
    dd = np.ascontiguousarray(np.asarray(D6, dtype=np.float64).reshape(6))
    gin = np.ascontiguousarray(np.asarray(gpre, dtype=np.float64))
    gout = np.zeros(cfg.q, dtype=np.float64)
    s = cfg.c_struct()
    _check(_tensor_load().oracle_collide_cell_tensor(ctypes.byref(s), _dp(dd), _dp(gin), _dp(gout)),
           "collide_cell_tensor")
    return gout


def collide_tensor(cfg: OracleConfig, D6, pre, nthreads: int = 1) -> np.ndarray:
    pre = _state(cfg, pre)
    post = np.zeros_like(pre)
    s = cfg.c_struct()
    _check(_tensor_load().oracle_collide_tensor(ctypes.byref(s), _dp(_tensor_field(cfg, D6)), _dp(pre),
                                                _dp(post), nthreads), "collide_tensor")
    return post


def run_tensor(cfg: OracleConfig, D6, nsteps: int, g=None, nthreads: int = 1) -> np.ndarray:
    """Advance with the tensor porosity control D6[6, N] (rows xx, yy, zz, xy, xz, yz)."""
    g = _state(cfg, g)
    s = cfg.c_struct()
    _check(_tensor_load().oracle_run_tensor(ctypes.byref(s), _dp(_tensor_field(cfg, D6)), int(nsteps),
                                            _dp(g), nthreads), "run_tensor")
    return g


def collide_adjoint_tensor(cfg: OracleConfig, D6, pre, post_bar, nthreads: int = 1):
    """(pre_bar, D_bar[6, N]) of one collision pass with the tensor control."""
    pre = _state(cfg, pre)
    pb = _state(cfg, post_bar)
    out = np.zeros_like(pre)
    Dbar = np.zeros((6, cfg.ncells))
    s = cfg.c_struct()
    _check(_tensor_load().oracle_collide_adjoint_tensor(ctypes.byref(s), _dp(_tensor_field(cfg, D6)), _dp(pre),
                                                        _dp(pb), _dp(out), _dp(Dbar), nthreads),
           "collide_adjoint_tensor")
    return out, Dbar


def gradient_tensor(cfg: OracleConfig, D6, nsteps: int, drho_bar, u_bar, every: int = 10,
                    nthreads: int = 1) -> np.ndarray:
    """d/dD6 (rows xx, yy, zz, xy, xz, yz) of <drho_bar, drho> + <u_bar, u> at the
    moments after nsteps from rest; an off-diagonal row is one variable that
    stands at two places of the symmetric matrix."""
    db = np.ascontiguousarray(np.asarray(drho_bar, dtype=np.float64).reshape(cfg.ncells))
    ub = np.ascontiguousarray(np.asarray(u_bar, dtype=np.float64).reshape(3, cfg.ncells))
    out = np.zeros((6, cfg.ncells))
    s = cfg.c_struct()
    _check(_tensor_load().oracle_gradient_tensor(ctypes.byref(s), _dp(_tensor_field(cfg, D6)), int(nsteps),
                                                 int(every), _dp(db), _dp(ub), _dp(out), nthreads),
           "gradient_tensor")
    return out


def _mask_load():
    lib = _load()
    if not getattr(lib, "_mask_ready", False):
        P = ctypes.POINTER
        D = P(ctypes.c_double)
        C = P(_Cfg)
        U8 = P(ctypes.c_ubyte)
        lib.oracle_stream_masked.argtypes = [C, U8, D, D, ctypes.c_int]
        lib.oracle_run_masked.argtypes = [C, U8, D, ctypes.c_int, D, ctypes.c_int]
        lib.oracle_observe_masked.argtypes = [C, U8, D, D, D, ctypes.c_int]
        lib._mask_ready = True
    return lib


def _mask(cfg: OracleConfig, mask):
    m = np.ascontiguousarray(np.asarray(mask).reshape(cfg.ncells).astype(np.uint8))
    return m, m.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))


def stream_masked(cfg: OracleConfig, mask, post, nthreads: int = 1) -> np.ndarray:
    """Pull streaming in a periodic box with solid cells (mask != 0)."""
    post = _state(cfg, post)
    pre = np.zeros_like(post)
    m, mp = _mask(cfg, mask)
    s = cfg.c_struct()
    _check(_mask_load().oracle_stream_masked(ctypes.byref(s), mp, _dp(post), _dp(pre), nthreads),
           "stream_masked")
    return pre


def run_masked(cfg: OracleConfig, mask, d, nsteps: int, g=None, nthreads: int = 1) -> np.ndarray:
    """Advance a periodic box with resolved solid cells (bounce-back links)."""
    g = _state(cfg, g)
    m, mp = _mask(cfg, mask)
    s = cfg.c_struct()
    _check(_mask_load().oracle_run_masked(ctypes.byref(s), mp, _dp(_field(cfg, d)), int(nsteps), _dp(g),
                                          nthreads), "run_masked")
    return g


def observe_masked(cfg: OracleConfig, mask, g, nthreads: int = 1):
    g = _state(cfg, g)
    drho = np.zeros(cfg.ncells)
    u = np.zeros((3, cfg.ncells))
    m, mp = _mask(cfg, mask)
    s = cfg.c_struct()
    _check(_mask_load().oracle_observe_masked(ctypes.byref(s), mp, _dp(g), _dp(drho), _dp(u), nthreads),
           "observe_masked")
    return drho, u


def collide_adjoint(cfg: OracleConfig, d, pre, post_bar, nthreads: int = 1):
    """(pre_bar, d_bar) of one collision pass."""
    pre = _state(cfg, pre)
    pb = _state(cfg, post_bar)
    out = np.zeros_like(pre)
    dbar = np.zeros(cfg.ncells)
    s = cfg.c_struct()
    _check(_adj_load().oracle_collide_adjoint(ctypes.byref(s), _dp(_field(cfg, d)), _dp(pre),
                                              _dp(pb), _dp(out), _dp(dbar), nthreads),
           "collide_adjoint")
    return out, dbar


def stream_adjoint(cfg: OracleConfig, post, pre_bar):
    post = _state(cfg, post)
    yb = _state(cfg, pre_bar)
    out = np.zeros_like(post)
    s = cfg.c_struct()
    _check(_adj_load().oracle_stream_adjoint(ctypes.byref(s), _dp(post), _dp(yb), _dp(out)),
           "stream_adjoint")
    return out


def moments_adjoint(cfg: OracleConfig, pre, drho_bar, u_bar):
    pre = _state(cfg, pre)
    db = np.ascontiguousarray(np.asarray(drho_bar, dtype=np.float64).reshape(cfg.ncells))
    ub = np.ascontiguousarray(np.asarray(u_bar, dtype=np.float64).reshape(3, cfg.ncells))
    out = np.zeros_like(pre)
    s = cfg.c_struct()
    _check(_adj_load().oracle_moments_adjoint(ctypes.byref(s), _dp(pre), _dp(db), _dp(ub),
                                              _dp(out)), "moments_adjoint")
    return out


def gradient(cfg: OracleConfig, d, nsteps: int, drho_bar, u_bar, every: int = 10,
             nthreads: int = 1) -> np.ndarray:
    """d/dd of <drho_bar, drho> + <u_bar, u> at the moments after nsteps from rest."""
    db = np.ascontiguousarray(np.asarray(drho_bar, dtype=np.float64).reshape(cfg.ncells))
    ub = np.ascontiguousarray(np.asarray(u_bar, dtype=np.float64).reshape(3, cfg.ncells))
    out = np.zeros(cfg.ncells)
    s = cfg.c_struct()
    _check(_adj_load().oracle_gradient(ctypes.byref(s), _dp(_field(cfg, d)), int(nsteps),
                                       int(every), _dp(db), _dp(ub), _dp(out), nthreads),
           "gradient")
    return out
