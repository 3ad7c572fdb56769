"""Shared helpers of the GPU parity tests (HIP path vs the FP64 oracle)."""
from __future__ import annotations

import numpy as np

from oracle import oracle as orc
from paper_1004_5059_amd import inputs
from paper_1004_5059_amd.tvlbm import LATTICE_ORDER, Solver


def rel_inf(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def make_pair(nx, ny, n=4, dtype="f64", tau=0.8, walls=False, wall_lo=(0.0, 1.0),
              wall_hi=(0.0, 1.0), collide=True, cfl=0.9, cfl_norm=0, compensated=True, variant=0,
              dy=None):
    """A GPU solver and an oracle grid with identical parameters."""
    s = Solver(nx, ny, n_gh=n, dtype=dtype, tau=tau, walls=walls, wall_lo=wall_lo,
               wall_hi=wall_hi, collide=collide, cfl=cfl, cfl_norm=cfl_norm,
               compensated=compensated, dy=dy)
    if variant:
        s.set_variant(variant)
    lat = orc.OracleLattice(n, LATTICE_ORDER[n], cfl=cfl, cfl_norm=cfl_norm)
    g = orc.OracleGrid(lat, nx, ny, tau=tau, collide=collide, walls=walls, wall_lo=wall_lo,
                       wall_hi=wall_hi, dy=dy)
    return s, g


def c0_inputs(nx=64, ny=64, q=16, seed=0):
    fields = inputs.shear_wave_fields(nx, ny, eps=0.01)
    noise = inputs.population_noise(q, ny, nx, amp=1e-4, seed=seed)
    return fields, noise


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)
