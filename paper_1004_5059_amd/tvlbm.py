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


class tvlbm_inst(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("wall_lo_ux", ctypes.c_double),
        ("wall_lo_T", ctypes.c_double),
        ("wall_hi_ux", ctypes.c_double),
        ("wall_hi_T", ctypes.c_double),
    ]


class tvlbm_batch_desc(ctypes.Structure):
    _fields_ = [
        ("n_gh", ctypes.c_int32),
        ("eq_order", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("compensated", ctypes.c_int32),
        ("cfl", ctypes.c_double),
        ("cfl_norm", ctypes.c_int32),
        ("n_inst", ctypes.c_int32),
        ("inst", ctypes.POINTER(tvlbm_inst)),
        ("arena_a", ctypes.c_void_p),
        ("arena_b", ctypes.c_void_p),
        ("stream", ctypes.c_void_p),
    ]


class tvlbm_batch_tuning(ctypes.Structure):
    _fields_ = [("prefetch", ctypes.c_int32), ("tail_active", ctypes.c_int32),
                ("tail_width", ctypes.c_int32), ("tail_rows", ctypes.c_int32),
                ("two_step", ctypes.c_int32), ("two_rows", ctypes.c_int32)]


class tvlbm_fv_desc(ctypes.Structure):
    _fields_ = [
        ("n_gh", ctypes.c_int32),
        ("eq_order", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("compensated", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("ld", ctypes.c_int64),
        ("dx", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("tau", ctypes.c_double),
        ("collide", ctypes.c_int32),
        ("y_bc", ctypes.c_int32),
        ("wall_lo_ux", ctypes.c_double),
        ("wall_lo_T", ctypes.c_double),
        ("wall_hi_ux", ctypes.c_double),
        ("wall_hi_T", ctypes.c_double),
        ("dy", ctypes.POINTER(ctypes.c_double)),
        ("f_a", ctypes.c_void_p),
        ("f_b", ctypes.c_void_p),
        ("omega", ctypes.c_void_p),
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
        "tvlbm_moments_static": [_vp, _vp, _vp, _vp],
        "tvlbm_residual": [_vp, _dp],
        "tvlbm_solve": [_vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, _i64p, _dp],
        "tvlbm_step_count": [_vp, _i64p],
        "tvlbm_lattice": [_vp, _dp, _dp, _dp, _dp],
        "tvlbm_lattice_table": [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                _dp, _dp, _dp, _dp],
        "tvlbm_save": [_vp, ctypes.c_char_p],
        "tvlbm_load": [_vp, ctypes.c_char_p],
        "tvlbm_ckpt_header": [ctypes.POINTER(tvlbm_desc), ctypes.c_int64, _vp, ctypes.c_int64],
        "tvlbm_ckpt_check": [_vp, ctypes.c_int64, ctypes.POINTER(tvlbm_desc), _i64p],
        "tvlbm_num_variants": [],
        "tvlbm_stream_copy": [_vp, _vp, ctypes.c_int64, _vp],
        "tvlbm_set_variant": [_vp, ctypes.c_int32],
        "tvlbm_steps_per_launch": [_vp, ctypes.POINTER(ctypes.c_int32)],
        "tvlbm_strerror": [ctypes.c_int],
        "tvlbm_last_error": [_vp],
        "tvlbm_batch_sizes": [ctypes.POINTER(tvlbm_batch_desc), _i64p, _i64p],
        "tvlbm_batch_init": [ctypes.POINTER(tvlbm_batch_desc), ctypes.POINTER(_vp)],
        "tvlbm_batch_destroy": [_vp],
        "tvlbm_batch_set_fields": [_vp, _vp],
        "tvlbm_batch_run": [_vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, _i64p, _dp],
        "tvlbm_batch_fields": [_vp, _vp],
        "tvlbm_batch_set_shape": [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
        "tvlbm_batch_set_tuning": [_vp, ctypes.c_void_p],
        "tvlbm_fv_init": [ctypes.c_void_p, ctypes.POINTER(_vp)],
        "tvlbm_fv_destroy": [_vp],
        "tvlbm_fv_set_fields": [_vp, _vp, _vp, _vp, _vp, _vp],
        "tvlbm_fv_step": [_vp, ctypes.c_int32],
        "tvlbm_fv_populations": [_vp, _vp],
        "tvlbm_fv_moments": [_vp, _vp, _vp, _vp, _vp, _dp],
        "tvlbm_fv_step_count": [_vp, _i64p],
        "tvlbm_fv_set_schedule": [_vp, ctypes.c_void_p],
        "tvlbm_fv_get_schedule": [_vp, ctypes.c_void_p],
        "tvlbm_fv_set_prandtl": [_vp, ctypes.c_double, ctypes.c_int32],
        "tvlbm_fv_set_wall_model": [_vp, ctypes.c_int32],
        "tvlbm_fv_set_x_ends": [_vp, ctypes.c_int32],
        "tvlbm_batch_get_tuning": [_vp, ctypes.c_void_p],
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


def tvlbm_stream_copy(src, dst, nbytes: int, stream=None):
    """Bandwidth probe: dst[:nbytes] = src[:nbytes] with the library's
    16-byte streaming copy kernel, on the given stream (or the null stream)."""
    st = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
    _check(lib().tvlbm_stream_copy(_ptr(src), _ptr(dst), int(nbytes), st))


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


def tvlbm_moments_static(ctx, fields=None, totals=None, flag=None):
    """Asynchronous, allocation-free moments: fields (device [4][ny][nx]),
    totals (device float64[4]) and flag (device int32[1]), each optional."""
    _check(lib().tvlbm_moments_static(ctx, _ptr(fields), _ptr(totals), _ptr(flag)), ctx)


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


def tvlbm_lattice_table(n_gh: int, eq_order: int, cfl: float = 0.9, cfl_norm: int = 0):
    """Host-only lattice tables: (xi [q][2], w [q], shift [q][2], lambda)."""
    q = n_gh * n_gh
    xi = (ctypes.c_double * (2 * q))()
    w = (ctypes.c_double * q)()
    sh = (ctypes.c_double * (2 * q))()
    lam = ctypes.c_double()
    _check(lib().tvlbm_lattice_table(n_gh, eq_order, cfl, cfl_norm, xi, w, sh, ctypes.byref(lam)))
    return (np.array(xi[:]).reshape(q, 2), np.array(w[:]), np.array(sh[:]).reshape(q, 2), lam.value)


def tvlbm_save(ctx, path: str):
    _check(lib().tvlbm_save(ctx, path.encode()), ctx)


def tvlbm_load(ctx, path: str):
    _check(lib().tvlbm_load(ctx, path.encode()), ctx)


TVLBM_CKPT_HEADER_BYTES = 128


def tvlbm_ckpt_header(desc: "tvlbm_desc", step: int) -> bytes:
    """Host only: the checkpoint header tvlbm_save writes for a context
    built from desc at `step`."""
    buf = ctypes.create_string_buffer(TVLBM_CKPT_HEADER_BYTES)
    _check(lib().tvlbm_ckpt_header(ctypes.byref(desc), int(step), buf, TVLBM_CKPT_HEADER_BYTES))
    return buf.raw


def tvlbm_ckpt_check(header: bytes, desc: "tvlbm_desc"):
    """Host only: the stored step count if tvlbm_load would accept a file
    with this header for a context built from desc, else None."""
    step = ctypes.c_int64(0)
    buf = ctypes.create_string_buffer(bytes(header), len(header))
    rc = lib().tvlbm_ckpt_check(buf, len(header), ctypes.byref(desc), ctypes.byref(step))
    if rc == TVLBM_EIO:
        return None
    _check(rc)
    return int(step.value)


def tvlbm_set_variant(ctx, v: int):
    _check(lib().tvlbm_set_variant(ctx, int(v)), ctx)


def tvlbm_steps_per_launch(ctx) -> int:
    k = ctypes.c_int32()
    _check(lib().tvlbm_steps_per_launch(ctx, ctypes.byref(k)), ctx)
    return k.value


# ------------------------------------------------------------- convenience --
class Solver:
    """One TVLBM grid on the current CUDA/HIP device.

    torch supplies the population buffers and the stream; every computation
    is a call into the HIP library.
    """

    def __init__(self, nx: int, ny: int, n_gh: int = 4, dtype: str = "f32", tau: float = 0.8,
                 cfl: float = 0.9, cfl_norm: int = TVLBM_CFL_EUCLID, collide: bool = True,
                 walls: bool = False, wall_lo=(0.0, 1.0), wall_hi=(0.0, 1.0),
                 compensated: bool = True, ld: int = 0, dy=None, device=None, stream=None):
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
        self._dy = None
        if dy is not None:
            self._dy = (ctypes.c_double * ny)(*[float(v) for v in dy])
            d.dy = ctypes.cast(self._dy, ctypes.POINTER(ctypes.c_double))
        else:
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
        t = self.torch.as_tensor(np.array(np.broadcast_to(a, shape)), dtype=self.tdtype)
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

    def steps_per_launch(self) -> int:
        return tvlbm_steps_per_launch(self.ctx)


# ----------------------------------------------------------------- batched --
def tvlbm_batch_sizes(desc: tvlbm_batch_desc):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().tvlbm_batch_sizes(ctypes.byref(desc), ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def tvlbm_batch_init(desc: tvlbm_batch_desc):
    h = _vp()
    _check(lib().tvlbm_batch_init(ctypes.byref(desc), ctypes.byref(h)))
    return h


def tvlbm_batch_destroy(h):
    _check(lib().tvlbm_batch_destroy(h))


def tvlbm_batch_set_fields(h, fields):
    _check(lib().tvlbm_batch_set_fields(h, _ptr(fields)))


def tvlbm_batch_run(h, n_inst: int, max_steps: int, tol: float, k_interval: int = 100):
    """(ok, steps, r): ok when every instance reached tol.  An instance that
    hit max_steps keeps its last residual; one whose state went non-finite
    (stopped at that check) has r = nan.  Other errors raise."""
    steps = (ctypes.c_int64 * n_inst)()
    r = (ctypes.c_double * n_inst)()
    rc = lib().tvlbm_batch_run(h, int(max_steps), float(tol), int(k_interval), steps, r)
    if rc not in (TVLBM_OK, TVLBM_ENOTCONVERGED, TVLBM_ENONFINITE):
        raise TvlbmError(rc, "batch run")
    return rc == TVLBM_OK, np.array(steps[:]), np.array(r[:])


def tvlbm_batch_fields(h, out, allow_nonfinite: bool = False):
    """allow_nonfinite: fill out even when some instance's fields are not
    finite (instead of raising ENONFINITE)."""
    rc = lib().tvlbm_batch_fields(h, _ptr(out))
    if rc == TVLBM_ENONFINITE and allow_nonfinite:
        return
    _check(rc)


def tvlbm_batch_set_shape(h, max_nx: int, width: int, rows: int):
    _check(lib().tvlbm_batch_set_shape(h, int(max_nx), int(width), int(rows)))


def tvlbm_batch_set_tuning(h, prefetch: int, tail_active: int, tail_width: int, tail_rows: int,
                           two_step: int = 1, two_rows: int = 8):
    t = tvlbm_batch_tuning(int(prefetch), int(tail_active), int(tail_width), int(tail_rows),
                           int(two_step), int(two_rows))
    _check(lib().tvlbm_batch_set_tuning(h, ctypes.byref(t)))


def tvlbm_batch_get_tuning(h):
    t = tvlbm_batch_tuning()
    _check(lib().tvlbm_batch_get_tuning(h, ctypes.byref(t)))
    return {"prefetch": t.prefetch, "tail_active": t.tail_active, "tail_width": t.tail_width,
            "tail_rows": t.tail_rows, "two_step": t.two_step, "two_rows": t.two_rows}


class BatchSolver:
    """Many walled channels (periodic in x) solved together on one GPU.

    instances: list of dicts with nx, ny, tau, and optionally u_bot, T_bot,
    u_top, T_top (bottom wall velocity/temperature, top wall ...)."""

    def __init__(self, instances, n_gh: int = 4, dtype: str = "f32", cfl: float = 0.9,
                 compensated: bool = True, device=None):
        import torch

        self.torch = torch
        self.device = torch.device(device or "cuda:0")
        self.n = len(instances)
        self.q = n_gh * n_gh
        self.tdtype = torch.float32 if dtype == "f32" else torch.float64
        arr = (tvlbm_inst * self.n)()
        for k, d in enumerate(instances):
            arr[k].nx, arr[k].ny = int(d["nx"]), int(d["ny"])
            arr[k].tau = float(d["tau"])
            arr[k].wall_lo_ux = float(d.get("u_bot", 0.0))
            arr[k].wall_lo_T = float(d.get("T_bot", 1.0))
            arr[k].wall_hi_ux = float(d.get("u_top", 0.0))
            arr[k].wall_hi_T = float(d.get("T_top", 1.0))
        self._arr = arr
        self.shapes = [(int(d["nx"]), int(d["ny"])) for d in instances]
        self.fld_off = np.concatenate([[0], np.cumsum([4 * nx * ny for nx, ny in self.shapes])])
        desc = tvlbm_batch_desc()
        desc.n_gh = n_gh
        desc.eq_order = LATTICE_ORDER[n_gh]
        desc.dtype = TVLBM_F32 if dtype == "f32" else TVLBM_F64
        desc.compensated = int(compensated)
        desc.cfl = cfl
        desc.cfl_norm = TVLBM_CFL_EUCLID
        desc.n_inst = self.n
        desc.inst = ctypes.cast(arr, ctypes.POINTER(tvlbm_inst))
        pop, fld = tvlbm_batch_sizes(desc)
        self.pop_elems, self.field_elems = pop, fld
        self.arena_a = torch.zeros(pop, dtype=self.tdtype, device=self.device)
        self.arena_b = torch.zeros(pop, dtype=self.tdtype, device=self.device)
        self.stream = torch.cuda.Stream(self.device)
        desc.arena_a = self.arena_a.data_ptr()
        desc.arena_b = self.arena_b.data_ptr()
        desc.stream = self.stream.cuda_stream
        self.desc = desc
        torch.cuda.synchronize()
        self.h = tvlbm_batch_init(desc)

    def close(self):
        if getattr(self, "h", None):
            tvlbm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_fields(self, fields):
        """fields: list of (rho, ux, uy, T) per instance (arrays [ny][nx] or
        scalars), or one packed array of length field_elems."""
        if isinstance(fields, (list, tuple)):
            parts = []
            for (nx, ny), f in zip(self.shapes, fields):
                parts.append(np.stack([np.broadcast_to(np.asarray(a, dtype=np.float64), (ny, nx))
                                       for a in f]).ravel())
            packed = np.concatenate(parts)
        else:
            packed = np.asarray(fields, dtype=np.float64).ravel()
        t = self.torch.as_tensor(packed, dtype=self.tdtype).to(self.device)
        self.torch.cuda.synchronize()
        tvlbm_batch_set_fields(self.h, t)
        self.stream.synchronize()

    def set_fields_device(self, packed):
        """packed: device tensor of field_elems values in the solver dtype."""
        self.torch.cuda.synchronize()
        tvlbm_batch_set_fields(self.h, packed)
        self.stream.synchronize()

    def set_shape(self, max_nx: int, width: int, rows: int):
        tvlbm_batch_set_shape(self.h, max_nx, width, rows)

    def set_tuning(self, prefetch: int = 1, tail_active: int = 0, tail_width: int = 64,
                   tail_rows: int = 1, two_step: int = 1, two_rows: int = 8):
        tvlbm_batch_set_tuning(self.h, prefetch, tail_active, tail_width, tail_rows, two_step,
                               two_rows)

    def tuning(self):
        return tvlbm_batch_get_tuning(self.h)

    def run(self, max_steps: int, tol: float = 1e-8, k_interval: int = 100):
        return tvlbm_batch_run(self.h, self.n, max_steps, tol, k_interval)

    def fields_packed(self, allow_nonfinite: bool = False):
        out = self.torch.empty(self.field_elems, dtype=self.tdtype, device=self.device)
        tvlbm_batch_fields(self.h, out, allow_nonfinite)
        return out

    def fields(self, allow_nonfinite: bool = False):
        """Per-instance [4][ny][nx] fields; allow_nonfinite: return them even
        if some instance went non-finite (its arrays then hold nan/inf)."""
        flat = self.fields_packed(allow_nonfinite).double().cpu().numpy()
        return [flat[self.fld_off[k]:self.fld_off[k + 1]].reshape(4, ny, nx)
                for k, (nx, ny) in enumerate(self.shapes)]


# ----------------------------------------------------- warm-start network --
class tvnet_desc(ctypes.Structure):
    _fields_ = [
        ("c_in", ctypes.c_int32),
        ("width", ctypes.c_int32),
        ("c_out", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("cols", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
    ]


_fp = ctypes.POINTER(ctypes.c_float)


def _tvnet_lib():
    L = lib()
    if not hasattr(L, "_tvnet_sig"):
        sig = {
            "tvnet_init": [ctypes.POINTER(tvnet_desc), ctypes.POINTER(_vp)],
            "tvnet_destroy": [_vp],
            "tvnet_num_params": [_vp, _i64p],
            "tvnet_set_params": [_vp, _fp],
            "tvnet_get_params": [_vp, _fp],
            "tvnet_forward": [_vp, _vp, _vp, ctypes.c_int32],
            "tvnet_backward": [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_double, _dp],
            "tvnet_get_grads": [_vp, _fp],
            "tvnet_adam_step": [_vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                ctypes.c_int32],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L._tvnet_sig = True
    return L


def tvnet_init(desc: tvnet_desc):
    h = _vp()
    _check(_tvnet_lib().tvnet_init(ctypes.byref(desc), ctypes.byref(h)))
    return h


def tvnet_destroy(h):
    _check(_tvnet_lib().tvnet_destroy(h))


def tvnet_num_params(h) -> int:
    n = ctypes.c_int64()
    _check(_tvnet_lib().tvnet_num_params(h, ctypes.byref(n)))
    return n.value


def tvnet_set_params(h, params: np.ndarray):
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check(_tvnet_lib().tvnet_set_params(h, p.ctypes.data_as(_fp)))


def tvnet_get_params(h, n: int) -> np.ndarray:
    p = np.zeros(n, dtype=np.float32)
    _check(_tvnet_lib().tvnet_get_params(h, p.ctypes.data_as(_fp)))
    return p


def tvnet_forward(h, x, y, batch: int):
    _check(_tvnet_lib().tvnet_forward(h, _ptr(x), _ptr(y), int(batch)))


def tvnet_backward(h, target, mask, batch: int, mask_sum: float) -> float:
    loss = ctypes.c_double()
    _check(_tvnet_lib().tvnet_backward(h, _ptr(target), _ptr(mask), int(batch), float(mask_sum),
                                       ctypes.byref(loss)))
    return loss.value


def tvnet_get_grads(h, n: int) -> np.ndarray:
    g = np.zeros(n, dtype=np.float32)
    _check(_tvnet_lib().tvnet_get_grads(h, g.ctypes.data_as(_fp)))
    return g


def tvnet_adam_step(h, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8, t: int = 1):
    _check(_tvnet_lib().tvnet_adam_step(h, lr, b1, b2, eps, int(t)))


class TvNet:
    """The warm-start network on the GPU; tensors are torch device tensors,
    channels last."""

    def __init__(self, c_in: int, height: int, cols: int, max_batch: int, c_out: int = 4,
                 device=None, stream=None):
        import torch

        self.torch = torch
        self.device = torch.device(device or "cuda:0")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        d = tvnet_desc()
        d.c_in, d.width, d.c_out = c_in, 32, c_out
        d.height, d.cols, d.max_batch = height, cols, max_batch
        d.stream = self.stream.cuda_stream
        self.c_in, self.c_out, self.H, self.W, self.max_batch = c_in, c_out, height, cols, max_batch
        self.h = tvnet_init(d)
        self.n_params = tvnet_num_params(self.h)
        self.t = 0

    def close(self):
        if getattr(self, "h", None):
            tvnet_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat):
        tvnet_set_params(self.h, flat)
        self.t = 0

    def params(self):
        return tvnet_get_params(self.h, self.n_params)

    def forward(self, x):
        B = x.shape[0]
        y = self.torch.empty((B, self.H, self.W, self.c_out), dtype=self.torch.float32, device=self.device)
        tvnet_forward(self.h, x.contiguous(), y, B)
        return y

    def backward(self, target, mask) -> float:
        B = target.shape[0]
        ms = float(mask.sum().item())
        return tvnet_backward(self.h, target.contiguous(), mask.contiguous(), B, ms)

    def grads(self):
        return tvnet_get_grads(self.h, self.n_params)

    def adam_step(self, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
        self.t += 1
        tvnet_adam_step(self.h, lr, b1, b2, eps, self.t)


# ------------------------------------------------------ finite volume ---
def tvlbm_fv_init(desc: tvlbm_fv_desc):
    h = _vp()
    _check(lib().tvlbm_fv_init(ctypes.byref(desc), ctypes.byref(h)))
    return h


def tvlbm_fv_destroy(h):
    _check(lib().tvlbm_fv_destroy(h))


def tvlbm_fv_set_fields(h, rho, ux, uy, T, noise=None):
    _check(lib().tvlbm_fv_set_fields(h, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T), _ptr(noise)))


def tvlbm_fv_step(h, nsteps: int):
    _check(lib().tvlbm_fv_step(h, int(nsteps)))


def tvlbm_fv_populations(h, out):
    _check(lib().tvlbm_fv_populations(h, _ptr(out)))


def tvlbm_fv_moments(h, rho=None, ux=None, uy=None, T=None):
    tot = (ctypes.c_double * 4)()
    _check(lib().tvlbm_fv_moments(h, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T), tot))
    return np.array(tot[:])


class tvlbm_fv_schedule(ctypes.Structure):
    _fields_ = [("fused", ctypes.c_int32), ("seg_rows", ctypes.c_int32),
                ("prefetch", ctypes.c_int32)]


def tvlbm_fv_set_schedule(h, fused: int, seg_rows: int = 0, prefetch: int = 1):
    s = tvlbm_fv_schedule(int(fused), int(seg_rows), int(prefetch))
    _check(lib().tvlbm_fv_set_schedule(h, ctypes.byref(s)))


def tvlbm_fv_get_schedule(h) -> dict:
    s = tvlbm_fv_schedule()
    _check(lib().tvlbm_fv_get_schedule(h, ctypes.byref(s)))
    return {"fused": s.fused, "seg_rows": s.seg_rows, "prefetch": s.prefetch}


def tvlbm_fv_set_prandtl(h, tau_g: float, pressure_scaled: bool = False):
    _check(lib().tvlbm_fv_set_prandtl(h, float(tau_g), int(pressure_scaled)))


TVLBM_FV_WALL_DIFFUSE, TVLBM_FV_WALL_SLIP_FREE = 0, 1


def tvlbm_fv_set_wall_model(h, model: int):
    _check(lib().tvlbm_fv_set_wall_model(h, int(model)))


TVLBM_FV_X_PERIODIC, TVLBM_FV_X_ZERO_GRADIENT = 0, 1


def tvlbm_fv_set_x_ends(h, mode: int):
    _check(lib().tvlbm_fv_set_x_ends(h, int(mode)))


def tvlbm_fv_step_count(h) -> int:
    k = ctypes.c_int64()
    _check(lib().tvlbm_fv_step_count(h, ctypes.byref(k)))
    return k.value


class FVSolver:
    """The paper's finite-volume update, eq.(FVLB), on a mesh uniform in x
    (spacing dx) with spacings dy in y; periodic or with diffuse-scattering
    wall points (eq.(FVLB2), eq.(IMPOSITION)).  dy: ny spacings (periodic,
    the last closes the period) or ny-1 (walls); None = all dx."""

    def __init__(self, nx: int, ny: int, n_gh: int = 4, dtype: str = "f32", dx: float = 1.0,
                 dt: float = 0.1, tau: float = 0.8, dy=None, walls: bool = False,
                 wall_lo=(0.0, 1.0), wall_hi=(0.0, 1.0), collide: bool = True,
                 compensated: bool = True, device=None, stream=None, eq_order: int | None = None):
        import torch

        self.torch = torch
        self.device = torch.device(device or "cuda:0")
        self.nx, self.ny, self.n, self.q = nx, ny, n_gh, n_gh * n_gh
        self.tdtype = torch.float32 if dtype == "f32" else torch.float64
        self.ld = ((nx + 63) // 64) * 64
        n_el = self.q * ny * self.ld
        self.f_a = torch.zeros(n_el, dtype=self.tdtype, device=self.device)
        self.f_b = torch.zeros(n_el, dtype=self.tdtype, device=self.device)
        self.om = torch.zeros(n_el, dtype=self.tdtype, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        d = tvlbm_fv_desc()
        d.n_gh, d.eq_order = n_gh, LATTICE_ORDER[n_gh] if eq_order is None else eq_order
        d.dtype = TVLBM_F32 if dtype == "f32" else TVLBM_F64
        d.compensated = int(compensated)
        d.nx, d.ny, d.ld = nx, ny, self.ld
        d.dx, d.dt, d.tau = dx, dt, tau
        d.collide = int(collide)
        d.y_bc = TVLBM_BC_DIFFUSE_WALLS if walls else TVLBM_BC_PERIODIC
        d.wall_lo_ux, d.wall_lo_T = wall_lo
        d.wall_hi_ux, d.wall_hi_T = wall_hi
        self._dy = None
        if dy is not None:
            self._dy = (ctypes.c_double * len(dy))(*[float(v) for v in dy])
            d.dy = ctypes.cast(self._dy, ctypes.POINTER(ctypes.c_double))
        d.f_a, d.f_b, d.omega = self.f_a.data_ptr(), self.f_b.data_ptr(), self.om.data_ptr()
        d.stream = self.stream.cuda_stream
        self.h = tvlbm_fv_init(d)

    def close(self):
        if getattr(self, "h", None):
            tvlbm_fv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a, shape):
        t = self.torch.as_tensor(np.ascontiguousarray(np.broadcast_to(a, shape)), dtype=self.tdtype)
        return t.to(self.device).contiguous()

    def set_fields(self, rho, ux, uy, T, noise=None):
        shp = (self.ny, self.nx)
        fl = [self._dev(a, shp) for a in (rho, ux, uy, T)]
        nz = None if noise is None else self._dev(noise, (self.q, self.ny, self.nx))
        tvlbm_fv_set_fields(self.h, *fl, nz)
        self.stream.synchronize()

    def step(self, n: int = 1):
        tvlbm_fv_step(self.h, n)

    def populations(self):
        out = self.torch.empty((self.q, self.ny, self.nx), dtype=self.tdtype, device=self.device)
        tvlbm_fv_populations(self.h, out)
        self.stream.synchronize()
        return out

    def moments(self):
        outs = [self.torch.empty((self.ny, self.nx), dtype=self.tdtype, device=self.device)
                for _ in range(4)]
        tot = tvlbm_fv_moments(self.h, *outs)
        return self.torch.stack(outs), tot

    @property
    def step_count(self) -> int:
        return tvlbm_fv_step_count(self.h)

    def set_schedule(self, fused: bool = True, seg_rows: int = 0, prefetch: bool = True):
        """fused: one pass per step (default) or the two-pass schedule;
        seg_rows: rows per wavefront of the fused pass (0 keeps it)."""
        tvlbm_fv_set_schedule(self.h, int(fused), seg_rows, int(prefetch))

    def schedule(self) -> dict:
        return tvlbm_fv_get_schedule(self.h)

    def set_prandtl(self, tau_g: float, pressure_scaled: bool = False):
        """Non-unit Prandtl number (eq.(FINAL)): tau_g > 0 adds the Pi term,
        0 removes it; pressure_scaled divides both relaxation times by the
        local pressure rho T."""
        tvlbm_fv_set_prandtl(self.h, tau_g, pressure_scaled)

    def set_wall_model(self, slip_free: bool):
        """Diffuse walls with the fixed wall equilibrium (False, default) or
        slip-free walls (True): the wall equilibrium is Newton-iterated so that
        the wall points carry the prescribed velocity and temperature."""
        tvlbm_fv_set_wall_model(self.h, TVLBM_FV_WALL_SLIP_FREE if slip_free else TVLBM_FV_WALL_DIFFUSE)

    def set_x_ends(self, zero_gradient: bool):
        """Periodic x (False, default) or zero-gradient (adiabatic) x ends."""
        tvlbm_fv_set_x_ends(self.h, TVLBM_FV_X_ZERO_GRADIENT if zero_gradient else TVLBM_FV_X_PERIODIC)
