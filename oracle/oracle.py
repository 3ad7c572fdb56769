"""Python view of the FP64 CPU oracle (``tvlbm_oracle.c``, and
``tvlbm_fv_oracle.c`` for the finite-volume update).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of the benchmark.  The product library never imports
it, and it imports nothing from the product package.

Every function here is argument marshalling around the C oracle; the
arithmetic lives in ``tvlbm_oracle.c`` (see its header for the passages of
the paper each part follows).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "tvlbm_oracle.c"), os.path.join(_HERE, "tvlbm_fv_oracle.c")]
_HDRS = [os.path.join(_HERE, "tvlbm_oracle.h"), os.path.join(_HERE, "tvlbm_fv_oracle.h")]
_LIB_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIB_DIR, "libtvlbm_oracle.so")

QMAX = 64
NMAX = 8


class Lattice(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int),
        ("q", ctypes.c_int),
        ("order", ctypes.c_int),
        ("x", ctypes.c_double * NMAX),
        ("wx", ctypes.c_double * NMAX),
        ("xi", (ctypes.c_double * 2) * QMAX),
        ("w", ctypes.c_double * QMAX),
        ("lam", ctypes.c_double),
        ("s", (ctypes.c_double * 2) * QMAX),
    ]


_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


class Grid(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int),
        ("ny", ctypes.c_int),
        ("tau", ctypes.c_double),
        ("collide", ctypes.c_int),
        ("walls", ctypes.c_int),
        ("ulo", ctypes.c_double),
        ("Tlo", ctypes.c_double),
        ("uhi", ctypes.c_double),
        ("Thi", ctypes.c_double),
        ("y", _dp),
        ("dy", _dp),
        ("yk_start", _ip),
        ("yk_src", _ip),
        ("yk_len", _dp),
        ("blo", _dp),
        ("ahi", _dp),
        ("glo", _dp),
        ("ghi", _dp),
        ("zlo", ctypes.c_double),
        ("zhi", ctypes.c_double),
        ("fw_lo", ctypes.c_double * QMAX),
        ("fw_hi", ctypes.c_double * QMAX),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, FP64, no contraction)."""
    os.makedirs(_LIB_DIR, exist_ok=True)
    newest = max(os.path.getmtime(f) for f in _SRCS + _HDRS)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
            "-shared", "-std=c11", "-Wall", "-o", tmp, *_SRCS, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        L = ctypes.POINTER(Lattice)
        G = ctypes.POINTER(Grid)
        _lib.orc_gauss_hermite.argtypes = [ctypes.c_int, _dp, _dp]
        _lib.orc_lattice_gh.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, L]
        _lib.orc_feq.argtypes = [L, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
        _lib.orc_feq.restype = None
        _lib.orc_moments.argtypes = [L, _dp, ctypes.c_long, _dp, _dp, _dp, _dp]
        _lib.orc_moments.restype = None
        _lib.orc_grid_init.argtypes = [L, G, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_double,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double]
        _lib.orc_grid_free.argtypes = [G]
        _lib.orc_grid_free.restype = None
        for name in ("orc_set_fields",):
            getattr(_lib, name).argtypes = [L, G, _dp, _dp, _dp, _dp, _dp, _dp]
            getattr(_lib, name).restype = None
        for name in ("orc_collide", "orc_stream", "orc_fields", "orc_totals"):
            getattr(_lib, name).argtypes = [L, G, _dp, _dp]
            getattr(_lib, name).restype = None
        _lib.orc_step.argtypes = [L, G, _dp, _dp, _dp]
        _lib.orc_step.restype = None
        _lib.orc_run.argtypes = [L, G, _dp, ctypes.c_int]
        _lib.orc_run.restype = None
        for name in ("orc_wall_incident", "orc_wall_emitted"):
            getattr(_lib, name).argtypes = [L, G, _dp, _dp, _dp]
            getattr(_lib, name).restype = None
        _lib.orc_residual.argtypes = [_dp, _dp, ctypes.c_long, ctypes.c_int]
        _lib.orc_residual.restype = ctypes.c_double
        _lib.orc_threads.restype = ctypes.c_int
        _lib.orc_set_threads.argtypes = [ctypes.c_int]
        FG = ctypes.POINTER(FVGrid)
        _lib.orc_fv_init.argtypes = [L, FG, ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double]
        _lib.orc_fv_free.argtypes = [FG]
        _lib.orc_fv_free.restype = None
        _lib.orc_fv_impose.argtypes = [L, FG, _dp]
        _lib.orc_fv_impose.restype = None
        _lib.orc_fv_set_fields.argtypes = [L, FG, _dp, _dp, _dp, _dp, _dp, _dp]
        _lib.orc_fv_set_fields.restype = None
        _lib.orc_fv_step.argtypes = [L, FG, _dp, _dp]
        _lib.orc_fv_step.restype = None
        _lib.orc_fv_run.argtypes = [L, FG, _dp, ctypes.c_int]
        _lib.orc_fv_run.restype = None
        _lib.orc_fv_dual.argtypes = [FG, ctypes.c_int]
        _lib.orc_fv_dual.restype = ctypes.c_double
        _lib.orc_fv_totals.argtypes = [L, FG, _dp, _dp]
        _lib.orc_fv_totals.restype = None
        _lib.orc_fv_set_prandtl.argtypes = [FG, ctypes.c_double, ctypes.c_int]
        _lib.orc_fv_set_prandtl.restype = None
        _lib.orc_fv_set_wall_model.argtypes = [FG, ctypes.c_int]
        _lib.orc_fv_set_wall_model.restype = None
        _lib.orc_fv_set_x_ends.argtypes = [FG, ctypes.c_int]
        _lib.orc_fv_set_x_ends.restype = None
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def gauss_hermite(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    if lib().orc_gauss_hermite(n, _p(x), _p(w)) != 0:
        raise ValueError("bad n")
    return x, w


class OracleLattice:
    """Tensor-product Gauss-Hermite velocity set (D2Q{n^2})."""

    def __init__(self, n: int, order: int, cfl: float = 0.9, cfl_norm: int = 0):
        self.c = Lattice()
        rc = lib().orc_lattice_gh(n, order, cfl, cfl_norm, ctypes.byref(self.c))
        if rc != 0:
            raise ValueError(f"invalid lattice n={n} order={order} cfl={cfl}")
        self.n, self.q, self.order = n, n * n, order
        self.xi = np.array([[self.c.xi[l][0], self.c.xi[l][1]] for l in range(self.q)])
        self.w = np.array([self.c.w[l] for l in range(self.q)])
        self.s = np.array([[self.c.s[l][0], self.c.s[l][1]] for l in range(self.q)])
        self.lam = self.c.lam
        self.x = np.array(self.c.x[:n])
        self.wx = np.array(self.c.wx[:n])

    def feq(self, rho, ux, uy, T) -> np.ndarray:
        out = np.zeros(self.q)
        lib().orc_feq(ctypes.byref(self.c), rho, ux, uy, T, _p(out))
        return out

    def moments(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64)
        r, ux, uy, T = (ctypes.c_double() for _ in range(4))
        lib().orc_moments(ctypes.byref(self.c), _p(f), 1, ctypes.byref(r), ctypes.byref(ux),
                          ctypes.byref(uy), ctypes.byref(T))
        return r.value, ux.value, uy.value, T.value


class OracleGrid:
    """A grid plus boundary set-up; f arrays are [q][ny][nx] float64."""

    def __init__(self, lat: OracleLattice, nx: int, ny: int, tau: float, dy=None, collide=True,
                 walls=False, wall_lo=(0.0, 1.0), wall_hi=(0.0, 1.0)):
        self.lat = lat
        self.nx, self.ny = nx, ny
        self.g = Grid()
        self._dy = None if dy is None else np.ascontiguousarray(dy, dtype=np.float64)
        rc = lib().orc_grid_init(ctypes.byref(lat.c), ctypes.byref(self.g), nx, ny,
                                 None if self._dy is None else _p(self._dy), tau, int(collide),
                                 int(walls), wall_lo[0], wall_lo[1], wall_hi[0], wall_hi[1])
        if rc != 0:
            lib().orc_grid_free(ctypes.byref(self.g))
            raise ValueError("invalid grid")
        self.dy = np.array([self.g.dy[j] for j in range(ny)])

    def __del__(self):
        try:
            lib().orc_grid_free(ctypes.byref(self.g))
        except Exception:
            pass

    @property
    def shape(self):
        return (self.lat.q, self.ny, self.nx)

    def _args(self):
        return ctypes.byref(self.lat.c), ctypes.byref(self.g)

    def set_fields(self, rho, ux, uy, T, noise=None) -> np.ndarray:
        fld = [np.ascontiguousarray(np.broadcast_to(a, (self.ny, self.nx)), dtype=np.float64)
               for a in (rho, ux, uy, T)]
        f = np.zeros(self.shape)
        nz = None if noise is None else _p(np.ascontiguousarray(noise, dtype=np.float64))
        lib().orc_set_fields(*self._args(), *[_p(a) for a in fld], nz, _p(f))
        return f

    def collide(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        out = np.zeros(self.shape)
        lib().orc_collide(*self._args(), _p(f), _p(out))
        return out

    def stream(self, fstar):
        fstar = np.ascontiguousarray(fstar, dtype=np.float64)
        out = np.zeros(self.shape)
        lib().orc_stream(*self._args(), _p(fstar), _p(out))
        return out

    def step(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        out = np.zeros(self.shape)
        work = np.zeros(self.shape)
        lib().orc_step(*self._args(), _p(f), _p(out), _p(work))
        return out

    def run(self, f, nsteps: int):
        f = np.array(f, dtype=np.float64, copy=True, order="C")
        lib().orc_run(*self._args(), _p(f), int(nsteps))
        return f

    def fields(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        out = np.zeros((4, self.ny, self.nx))
        lib().orc_fields(*self._args(), _p(f), _p(out))
        return out

    def totals(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        out = np.zeros(4)
        lib().orc_totals(*self._args(), _p(f), _p(out))
        return out

    def wall_incident(self, fstar):
        fstar = np.ascontiguousarray(fstar, dtype=np.float64)
        lo, hi = np.zeros(self.nx), np.zeros(self.nx)
        lib().orc_wall_incident(*self._args(), _p(fstar), _p(lo), _p(hi))
        return lo, hi

    def wall_emitted(self, fstar):
        fstar = np.ascontiguousarray(fstar, dtype=np.float64)
        lo, hi = np.zeros(self.nx), np.zeros(self.nx)
        lib().orc_wall_emitted(*self._args(), _p(fstar), _p(lo), _p(hi))
        return lo, hi


class FVGrid(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int),
        ("ny", ctypes.c_int),
        ("dx", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("tau", ctypes.c_double),
        ("collide", ctypes.c_int),
        ("walls", ctypes.c_int),
        ("ulo", ctypes.c_double),
        ("Tlo", ctypes.c_double),
        ("uhi", ctypes.c_double),
        ("Thi", ctypes.c_double),
        ("dy", _dp),
        ("emit_lo", ctypes.c_double * QMAX),
        ("emit_hi", ctypes.c_double * QMAX),
        ("tau_g", ctypes.c_double),
        ("pscale", ctypes.c_int),
        ("slip_free", ctypes.c_int),
        ("x_open", ctypes.c_int),
        ("nr_last", ctypes.c_int),
    ]


class OracleFVGrid:
    """Mesh for the finite-volume update (``tvlbm_fv_oracle.h``); f arrays
    are [q][ny][nx] float64 over the mesh points."""

    def __init__(self, lat: OracleLattice, nx: int, ny: int, dx: float, dt: float, tau: float,
                 dy=None, collide=True, walls=False, wall_lo=(0.0, 1.0), wall_hi=(0.0, 1.0),
                 tau_g: float = 0.0, pscale: bool = False, slip_free: bool = False,
                 x_open: bool = False):
        self.lat = lat
        self.nx, self.ny = nx, ny
        self.g = FVGrid()
        self._dy = None if dy is None else np.ascontiguousarray(dy, dtype=np.float64)
        rc = lib().orc_fv_init(ctypes.byref(lat.c), ctypes.byref(self.g), nx, ny, dx,
                               None if self._dy is None else _p(self._dy), dt, tau, int(collide),
                               int(walls), wall_lo[0], wall_lo[1], wall_hi[0], wall_hi[1])
        if rc != 0:
            lib().orc_fv_free(ctypes.byref(self.g))
            raise ValueError("invalid finite-volume mesh")
        self.dual = np.array([lib().orc_fv_dual(ctypes.byref(self.g), j) for j in range(ny)])
        lib().orc_fv_set_prandtl(ctypes.byref(self.g), float(tau_g), int(pscale))
        lib().orc_fv_set_wall_model(ctypes.byref(self.g), int(slip_free))
        lib().orc_fv_set_x_ends(ctypes.byref(self.g), int(x_open))

    def __del__(self):
        try:
            lib().orc_fv_free(ctypes.byref(self.g))
        except Exception:
            pass

    @property
    def shape(self):
        return (self.lat.q, self.ny, self.nx)

    def _args(self):
        return ctypes.byref(self.lat.c), ctypes.byref(self.g)

    def set_fields(self, rho, ux, uy, T, noise=None) -> np.ndarray:
        fld = [np.ascontiguousarray(np.broadcast_to(a, (self.ny, self.nx)), dtype=np.float64)
               for a in (rho, ux, uy, T)]
        f = np.zeros(self.shape)
        nz = None if noise is None else _p(np.ascontiguousarray(noise, dtype=np.float64))
        lib().orc_fv_set_fields(*self._args(), *[_p(a) for a in fld], nz, _p(f))
        return f

    def impose(self, f):
        f = np.array(f, dtype=np.float64, copy=True, order="C")
        lib().orc_fv_impose(*self._args(), _p(f))
        return f

    def step(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        out = np.zeros(self.shape)
        lib().orc_fv_step(*self._args(), _p(f), _p(out))
        return out

    def run(self, f, nsteps: int):
        f = np.array(f, dtype=np.float64, copy=True, order="C")
        lib().orc_fv_run(*self._args(), _p(f), int(nsteps))
        return f

    def totals(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        out = np.zeros(4)
        lib().orc_fv_totals(*self._args(), _p(f), _p(out))
        return out

    def fields(self, f):
        """(rho, ux, uy, T) at every mesh point, [4][ny][nx]."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        out = np.zeros((4, self.ny, self.nx))
        for j in range(self.ny):
            for i in range(self.nx):
                out[:, j, i] = self.lat.moments(np.ascontiguousarray(f[:, j, i]))
        return out


def residual(q: np.ndarray, qprev: np.ndarray, K: int) -> float:
    q = np.ascontiguousarray(q, dtype=np.float64).ravel()
    qprev = np.ascontiguousarray(qprev, dtype=np.float64).ravel()
    return lib().orc_residual(_p(q), _p(qprev), q.size, int(K))


def threads() -> int:
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (timing only)."""
    lib().orc_set_threads(int(n))
