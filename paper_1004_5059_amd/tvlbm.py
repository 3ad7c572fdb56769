"""Python binding of the TVLBM C ABI (include/tvlbm.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``_lib/libtvlbm.so``.  The functions keep the C names; ``Solver``
adds torch-owned device buffers and the current torch stream.  If the built
library is missing, loading fails loudly -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libtvlbm.so")

TVLBM_OK = 0
TVLBM_EINVAL = -1
TVLBM_EHIP = -2
TVLBM_ENOMEM = -3
TVLBM_ENONFINITE = -4
TVLBM_EUNSUPPORTED = -5
TVLBM_ENOTCONVERGED = -6
TVLBM_EIO = -7

TVLBM_F32 = 0
TVLBM_F64 = 1
TVLBM_CFL_EUCLID = 0
TVLBM_CFL_COMPONENT = 1
TVLBM_BC_PERIODIC = 0
TVLBM_BC_DIFFUSE_WALLS = 1

LATTICE_ORDER = {3: 2, 4: 3, 6: 4}  # Gauss-Hermite points -> equilibrium order


class tvlbm_desc(ctypes.Structure):
    _fields_ = [
        ("n_gh", ctypes.c_int32),
        ("eq_order", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("cfl_norm", ctypes.c_int32),
        ("ld", ctypes.c_int64),
        ("tau", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("collide", ctypes.c_int32),
        ("y_bc", ctypes.c_int32),
        ("compensated", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("wall_lo_ux", ctypes.c_double),
        ("wall_lo_T", ctypes.c_double),
        ("wall_hi_ux", ctypes.c_double),
        ("wall_hi_T", ctypes.c_double),
        ("dy", ctypes.POINTER(ctypes.c_double)),
        ("f_a", ctypes.c_void_p),
        ("f_b", ctypes.c_void_p),
        ("stream", ctypes.c_void_p),
    ]


class TvlbmError(RuntimeError):
    def __init__(self, code: int, detail: str = ""):
        self.code = code
        super().__init__(f"tvlbm error {code} ({tvlbm_strerror(code)}): {detail}")


_lib = None
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)


def lib():
    """Load the built HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"TVLBM HIP library not built: {LIB_PATH} missing "
                           "(run __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "tvlbm_init": [ctypes.POINTER(tvlbm_desc), ctypes.POINTER(_vp)],
        "tvlbm_destroy": [_vp],
        "tvlbm_set_fields": [_vp, _vp, _vp, _vp, _vp, _vp],
        "tvlbm_set_populations": [_vp, _vp],
        "tvlbm_step": [_vp, ctypes.c_int32],
        "tvlbm_populations": [_vp, _vp],
        "tvlbm_post_collision": [_vp, _vp],
        "tvlbm_moments": [_vp, _vp, _vp, _vp, _vp, _dp],
        "tvlbm_residual": [_vp, _dp],
        "tvlbm_solve": [_vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, _i64p, _dp],
        "tvlbm_step_count": [_vp, _i64p],
        "tvlbm_lattice": [_vp, _dp, _dp, _dp, _dp],
        "tvlbm_save": [_vp, ctypes.c_char_p],
        "tvlbm_load": [_vp, ctypes.c_char_p],
        "tvlbm_num_variants": [],
        "tvlbm_set_variant": [_vp, ctypes.c_int32],
        "tvlbm_strerror": [ctypes.c_int],
        "tvlbm_last_error": [_vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.tvlbm_strerror.restype = ctypes.c_char_p
    L.tvlbm_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _ptr(x):
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return ctypes.c_void_p(x.data_ptr())
    return ctypes.c_void_p(int(x))


def _check(rc: int, ctx=None):
    if rc != TVLBM_OK:
        detail = tvlbm_last_error(ctx) if ctx else ""
        raise TvlbmError(rc, detail)


# ----------------------------------------------------- same-name wrappers --
def tvlbm_strerror(code: int) -> str:
    return lib().tvlbm_strerror(code).decode()


def tvlbm_last_error(ctx) -> str:
    return lib().tvlbm_last_error(ctx).decode()


def tvlbm_num_variants() -> int:
    return lib().tvlbm_num_variants()


def tvlbm_init(desc: tvlbm_desc):
    ctx = _vp()
    _check(lib().tvlbm_init(ctypes.byref(desc), ctypes.byref(ctx)))
    return ctx


def tvlbm_destroy(ctx):
    _check(lib().tvlbm_destroy(ctx))


def tvlbm_set_fields(ctx, rho, ux, uy, T, noise=None):
    _check(lib().tvlbm_set_fields(ctx, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T), _ptr(noise)), ctx)


def tvlbm_set_populations(ctx, f):
    _check(lib().tvlbm_set_populations(ctx, _ptr(f)), ctx)


def tvlbm_step(ctx, nsteps: int):
    _check(lib().tvlbm_step(ctx, int(nsteps)), ctx)


def tvlbm_populations(ctx, out):
    _check(lib().tvlbm_populations(ctx, _ptr(out)), ctx)


def tvlbm_post_collision(ctx, out):
    _check(lib().tvlbm_post_collision(ctx, _ptr(out)), ctx)


def tvlbm_moments(ctx, rho=None, ux=None, uy=None, T=None, check=True):
    tot = (ctypes.c_double * 4)()
    rc = lib().tvlbm_moments(ctx, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T), tot)
    if check:
        _check(rc, ctx)
    return (np.array(tot[:]), rc) if not check else np.array(tot[:])


def tvlbm_residual(ctx) -> float:
    r = ctypes.c_double()
    _check(lib().tvlbm_residual(ctx, ctypes.byref(r)), ctx)
    return r.value


def tvlbm_solve(ctx, max_steps: int, tol: float, k_interval: int = 100):
    steps = ctypes.c_int64()
    r = ctypes.c_double()
    rc = lib().tvlbm_solve(ctx, int(max_steps), float(tol), int(k_interval), ctypes.byref(steps),
                           ctypes.byref(r))
    if rc not in (TVLBM_OK, TVLBM_ENOTCONVERGED):
        _check(rc, ctx)
    return rc == TVLBM_OK, steps.value, r.value


def tvlbm_step_count(ctx) -> int:
    k = ctypes.c_int64()
    _check(lib().tvlbm_step_count(ctx, ctypes.byref(k)), ctx)
    return k.value


def tvlbm_lattice(ctx, q: int):
    xi = (ctypes.c_double * (2 * q))()
    w = (ctypes.c_double * q)()
    sh = (ctypes.c_double * (2 * q))()
    lam = ctypes.c_double()
    _check(lib().tvlbm_lattice(ctx, xi, w, sh, ctypes.byref(lam)), ctx)
    return (np.array(xi[:]).reshape(q, 2), np.array(w[:]), np.array(sh[:]).reshape(q, 2), lam.value)


def tvlbm_save(ctx, path: str):
    _check(lib().tvlbm_save(ctx, path.encode()), ctx)


def tvlbm_load(ctx, path: str):
    _check(lib().tvlbm_load(ctx, path.encode()), ctx)


def tvlbm_set_variant(ctx, v: int):
    _check(lib().tvlbm_set_variant(ctx, int(v)), ctx)


# ------------------------------------------------------------- convenience --
class Solver:
    """One TVLBM grid on the current CUDA/HIP device.

    torch supplies the population buffers and the stream; every computation
    is a call into the HIP library.
    """

    def __init__(self, nx: int, ny: int, n_gh: int = 4, dtype: str = "f32", tau: float = 0.8,
                 cfl: float = 0.9, cfl_norm: int = TVLBM_CFL_EUCLID, collide: bool = True,
                 walls: bool = False, wall_lo=(0.0, 1.0), wall_hi=(0.0, 1.0),
                 compensated: bool = True, ld: int = 0, device=None, stream=None):
        import torch

        self.torch = torch
        self.device = torch.device(device or "cuda:0")
        self.nx, self.ny, self.n, self.q = nx, ny, n_gh, n_gh * n_gh
        self.tdtype = torch.float32 if dtype == "f32" else torch.float64
        self.ld = ld if ld else ((nx + 63) // 64) * 64
        n_el = self.q * ny * self.ld
        self.f_a = torch.zeros(n_el, dtype=self.tdtype, device=self.device)
        self.f_b = torch.zeros(n_el, dtype=self.tdtype, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        d = tvlbm_desc()
        d.n_gh = n_gh
        d.eq_order = LATTICE_ORDER[n_gh]
        d.dtype = TVLBM_F32 if dtype == "f32" else TVLBM_F64
        d.nx, d.ny = nx, ny
        d.cfl_norm = cfl_norm
        d.ld = self.ld
        d.tau = tau
        d.cfl = cfl
        d.collide = int(collide)
        d.y_bc = TVLBM_BC_DIFFUSE_WALLS if walls else TVLBM_BC_PERIODIC
        d.compensated = int(compensated)
        d.wall_lo_ux, d.wall_lo_T = wall_lo
        d.wall_hi_ux, d.wall_hi_T = wall_hi
        d.dy = None
        d.f_a = self.f_a.data_ptr()
        d.f_b = self.f_b.data_ptr()
        d.stream = self.stream.cuda_stream
        self.desc = d
        self.ctx = tvlbm_init(d)

    def close(self):
        if getattr(self, "ctx", None):
            tvlbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a, shape):
        t = self.torch.as_tensor(np.ascontiguousarray(np.broadcast_to(a, shape)), dtype=self.tdtype)
        return t.to(self.device)

    def set_fields(self, rho, ux, uy, T, noise=None):
        shp = (self.ny, self.nx)
        fl = [self._dev(a, shp) for a in (rho, ux, uy, T)]
        nz = None if noise is None else self._dev(noise, (self.q, self.ny, self.nx))
        tvlbm_set_fields(self.ctx, *fl, nz)
        self.stream.synchronize()

    def set_populations(self, f):
        t = self._dev(f, (self.q, self.ny, self.nx))
        tvlbm_set_populations(self.ctx, t)
        self.stream.synchronize()

    def step(self, n: int = 1):
        tvlbm_step(self.ctx, n)

    def populations(self):
        out = self.torch.empty((self.q, self.ny, self.nx), dtype=self.tdtype, device=self.device)
        tvlbm_populations(self.ctx, out)
        return out

    def post_collision(self):
        out = self.torch.empty((self.q, self.ny, self.nx), dtype=self.tdtype, device=self.device)
        tvlbm_post_collision(self.ctx, out)
        return out

    def moments(self):
        """(fields [4][ny][nx] tensor: rho, ux, uy, T; totals M, Px, Py, E)."""
        f = self.torch.empty((4, self.ny, self.nx), dtype=self.tdtype, device=self.device)
        tot = tvlbm_moments(self.ctx, f[0], f[1], f[2], f[3])
        return f, tot

    def residual(self) -> float:
        return tvlbm_residual(self.ctx)

    def solve(self, max_steps: int, tol: float, k_interval: int = 100):
        return tvlbm_solve(self.ctx, max_steps, tol, k_interval)

    @property
    def step_count(self) -> int:
        return tvlbm_step_count(self.ctx)

    def lattice(self):
        return tvlbm_lattice(self.ctx, self.q)

    def set_variant(self, v: int):
        tvlbm_set_variant(self.ctx, v)
