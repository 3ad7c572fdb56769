"""Checkpoint header (format 2) on the CPU: the library's own header builder
and checker (the code tvlbm_save and tvlbm_load use), no device work.  A
header must accept the descriptor it was written for and refuse any change
to a field that alters the arithmetic of a step."""
import ctypes
import os
import struct

import numpy as np
import pytest

from paper_1004_5059_amd import inputs, tvlbm as T

pytestmark = pytest.mark.skipif(not os.path.exists(T.LIB_PATH), reason="library not built")

DY = inputs.refined_wall_rows(h=24, band=4, ratio=2)  # 32 rows


def _desc(**kw):
    d = T.tvlbm_desc()
    base = dict(n_gh=4, eq_order=3, dtype=T.TVLBM_F32, nx=40, ny=len(DY), cfl_norm=T.TVLBM_CFL_EUCLID,
                ld=0, tau=0.7, cfl=0.9, collide=1, y_bc=T.TVLBM_BC_DIFFUSE_WALLS, compensated=1,
                wall_lo_ux=0.0, wall_lo_T=1.0, wall_hi_ux=0.05, wall_hi_T=1.1)
    base.update(kw)
    dy = base.pop("dy", DY)
    for k, v in base.items():
        setattr(d, k, v)
    if dy is not None:
        arr = np.ascontiguousarray(dy, dtype=np.float64)
        d._dy_keep = arr  # keep the row heights alive while the descriptor is used
        d.dy = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return d


def test_header_accepts_its_own_descriptor_and_returns_the_step():
    h = T.tvlbm_ckpt_header(_desc(), 12345)
    assert len(h) == T.TVLBM_CKPT_HEADER_BYTES
    assert h[:8] == b"TVLBMCK2"
    assert T.tvlbm_ckpt_check(h, _desc()) == 12345


@pytest.mark.parametrize("change", [
    dict(cfl_norm=T.TVLBM_CFL_COMPONENT),
    dict(wall_lo_ux=0.01), dict(wall_lo_T=1.01), dict(wall_hi_ux=0.04), dict(wall_hi_T=1.2),
    dict(dy=np.where(np.arange(len(DY)) == 7, 0.75, DY)),  # one row height
    dict(dy=None, ny=len(DY)),  # unit rows instead of the refined table
    dict(compensated=0),
    dict(tau=0.7000000001), dict(cfl=0.8), dict(nx=41), dict(ld=128),
    dict(n_gh=6, eq_order=4), dict(dtype=T.TVLBM_F64), dict(collide=0),
    dict(y_bc=T.TVLBM_BC_PERIODIC),
])
def test_header_refuses_a_changed_descriptor(change):
    h = T.tvlbm_ckpt_header(_desc(), 7)
    assert T.tvlbm_ckpt_check(h, _desc(**change)) is None


def test_periodic_grids_ignore_wall_values_and_f64_ignores_compensation():
    per = dict(y_bc=T.TVLBM_BC_PERIODIC, dy=None)
    h = T.tvlbm_ckpt_header(_desc(**per), 3)
    assert T.tvlbm_ckpt_check(h, _desc(wall_lo_T=2.0, wall_hi_ux=-0.3, **per)) == 3
    h = T.tvlbm_ckpt_header(_desc(dtype=T.TVLBM_F64, compensated=1), 4)
    assert T.tvlbm_ckpt_check(h, _desc(dtype=T.TVLBM_F64, compensated=0)) == 4


def test_header_records_the_fields_at_their_documented_offsets():
    h = T.tvlbm_ckpt_header(_desc(), 99)
    magic, version, n_gh, eq, dt, nx, ny, ybc, col, norm, comp, _pad = struct.unpack_from("<8s11i", h, 0)
    assert (magic, version, n_gh, eq, dt, nx, ny) == (b"TVLBMCK2", 2, 4, 3, T.TVLBM_F32, 40, len(DY))
    assert (ybc, col, norm, comp) == (T.TVLBM_BC_DIFFUSE_WALLS, 1, T.TVLBM_CFL_EUCLID, 1)
    ld, step, tau, cfl, lo_u, lo_T, hi_u, hi_T, rh = struct.unpack_from("<2q6dQ", h, 56)
    assert (ld, step) == (64, 99)
    assert (tau, cfl, lo_u, lo_T, hi_u, hi_T) == (0.7, 0.9, 0.0, 1.0, 0.05, 1.1)
    # FNV-1a over the row heights' bytes, recomputed here
    fnv = 1469598103934665603
    for byte in np.ascontiguousarray(DY, dtype="<f8").tobytes():
        fnv = ((fnv ^ byte) * 1099511628211) % (1 << 64)
    assert rh == fnv
    assert struct.unpack_from("<Q", T.tvlbm_ckpt_header(_desc(dy=None), 0), 120)[0] == 0


def test_format_one_and_truncated_headers_are_refused():
    h = bytearray(T.tvlbm_ckpt_header(_desc(), 5))
    old = bytes(h[:8].replace(b"TVLBMCK2", b"TVLBMCK1")) + bytes(h[8:])
    assert T.tvlbm_ckpt_check(old, _desc()) is None
    assert T.tvlbm_ckpt_check(bytes(h[:100]), _desc()) is None
