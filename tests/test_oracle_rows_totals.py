"""Pins of the oracle's non-uniform-row remap, its wall geometry and its
conserved totals against values fixed independently of its code.

* Rows of one height h (the rectangular meshes of Sec. III, refined in y):
  a displacement of s cells is s/h rows, so a Fourier mode in the row index
  must be multiplied by the closed-form symbol of a shift by s/h rows --
  (1 - phi) e^{-i k m} + phi e^{-i k (m+1)} with m + phi = s/h -- which
  spreads over two rows and, once |s|/h > 1, moves past the neighbouring
  row.  A remap that measured the displacement in rows of the finest height,
  or in coarse cells on a fine mesh, fails it.
* A 4-row periodic mesh of two heights (0.5, 0.5, 1, 1): the remap matrix of
  each D2Q16 displacement, derived by hand below from the interval overlaps,
  entry by entry.
* The same mesh with diffuse walls: the lengths of the shifted rows that
  cross each wall, and the split of the emitted interval [0, s] over the
  first two rows.
* Totals (Sec. II): for cells at equilibrium, M = rho A, P = rho u A and
  E = (D/2 rho T + 1/2 rho |u|^2) A with D = 2, summed over rows of
  different areas A = n_x dy_j.
* The NumPy mini-oracle (oracle/mini.py, a second implementation built
  differently) agrees with the C oracle step by step.
"""
import math

import numpy as np
import pytest

from oracle import mini
from paper_1004_5059_amd import inputs


def _unit_response(orc, lat, dy, l, walls=False):
    """Columns of the y remap matrix of population l on a 1-column grid:
    out[k, j] = value landing in row k from a unit value in source row j."""
    ny = len(dy)
    g = orc.OracleGrid(lat, 1, ny, tau=1.0, dy=dy, collide=False, walls=walls)
    M = np.zeros((ny, ny))
    for j in range(ny):
        f = np.zeros((lat.q, ny, 1))
        f[l, j, 0] = 1.0
        M[:, j] = g.stream(f)[l, :, 0]
    return M


# --------------------------------------------------- uniform fine rows --
@pytest.mark.parametrize("n,order", [(4, 3), (6, 4)])
@pytest.mark.parametrize("h", [0.5, 0.25])
def test_fine_rows_shift_by_s_over_h_rows(orc, n, order, h):
    lat = orc.OracleLattice(n, order)
    nx, ny = 6, 24
    g = orc.OracleGrid(lat, nx, ny, tau=1.0, dy=np.full(ny, h), collide=False)
    for mx, my in ((0, 1), (1, 3), (2, -5)):
        kx, ky = 2 * np.pi * mx / nx, 2 * np.pi * my / ny
        ph = kx * np.arange(nx)[None, :] + ky * np.arange(ny)[:, None]
        fc = np.broadcast_to(np.cos(ph), g.shape).copy()
        fs = np.broadcast_to(np.sin(ph), g.shape).copy()
        oc, os_ = g.stream(fc), g.stream(fs)
        for l in range(lat.q):
            sx, sy = lat.s[l]
            symx = (1 - abs(sx)) + abs(sx) * np.exp(-1j * kx * np.sign(sx))
            r = sy / h  # displacement in rows
            m = math.floor(r)
            phi = r - m
            symy = (1 - phi) * np.exp(-1j * ky * m) + phi * np.exp(-1j * ky * (m + 1))
            np.testing.assert_allclose(oc[l] + 1j * os_[l], symx * symy * np.exp(1j * ph),
                                       atol=2e-14, err_msg=f"l={l} s={sx, sy} h={h}")


def test_fine_rows_reach_past_the_next_row(orc):
    """On rows of height 1/4 the outer D2Q16 displacement 0.6364 is 2.55
    rows: a unit value in row 0 lands in rows 2 and 3 only."""
    lat = orc.OracleLattice(4, 3)
    l = next(l for l in range(lat.q) if lat.s[l, 1] > 0.6)
    M = _unit_response(orc, lat, np.full(8, 0.25), l)
    r = lat.s[l, 1] / 0.25
    expect = np.zeros(8)
    expect[2], expect[3] = 1 - (r - 2), r - 2
    np.testing.assert_allclose(M[:, 0], expect, atol=1e-15)


# ----------------------------------------- two heights: matrices by hand --
DY4 = np.array([0.5, 0.5, 1.0, 1.0])


def _hand_matrix(s):
    """Remap matrix M[k, j] of the periodic rows (0.5, 0.5, 1, 1) (edges
    0, 0.5, 1, 2, 3) for a displacement s, from the overlaps of [y_j + s,
    y_{j+1} + s] (mod 3) with row k, divided by dy_k; worked out by hand for
    the four ranges the D2Q16 displacements fall in."""
    M = np.zeros((4, 4))
    if 0 < s < 0.5:
        M[0] = [1 - 2 * s, 0, 0, 2 * s]
        M[1] = [2 * s, 1 - 2 * s, 0, 0]
        M[2] = [0, s, 1 - s, 0]
        M[3] = [0, 0, s, 1 - s]
    elif 0.5 < s < 1:
        M[0] = [0, 0, 0, 1]
        M[1] = [2 * (1 - s), 0, 0, 2 * s - 1]
        M[2] = [s - 0.5, 0.5, 1 - s, 0]
        M[3] = [0, 0, s, 1 - s]
    elif -0.5 < s < 0:
        a = -s
        M[0] = [1 - 2 * a, 2 * a, 0, 0]
        M[1] = [0, 1 - 2 * a, 2 * a, 0]
        M[2] = [0, 0, 1 - a, a]
        M[3] = [a, 0, 0, 1 - a]
    elif -1 < s < -0.5:
        a = -s
        M[0] = [0, 2 * (1 - a), 2 * a - 1, 0]
        M[1] = [0, 0, 1, 0]
        M[2] = [0, 0, 1 - a, a]
        M[3] = [0.5, a - 0.5, 0, 1 - a]
    else:
        raise ValueError(s)
    return M


def test_two_height_rows_match_hand_matrices(orc):
    lat = orc.OracleLattice(4, 3)
    seen = set()
    for l in range(lat.q):
        s = lat.s[l, 1]
        if s in seen:
            continue
        seen.add(s)
        M = _unit_response(orc, lat, DY4, l)
        np.testing.assert_allclose(M, _hand_matrix(s), atol=2e-15, err_msg=f"s = {s}")
        # each source row's mass goes somewhere: sum_k dy_k M[k, j] = dy_j
        np.testing.assert_allclose(DY4 @ M, DY4, atol=2e-15)
    assert len(seen) == 4


def test_two_height_rows_wall_crossing_lengths(orc):
    """Walls at y = 0 and y = 3 on the rows (0.5, 0.5, 1, 1): a unit value in
    row j of a population moving down by a crosses the bottom wall over the
    length of [y_j - a, y_{j+1} - a] below 0 (0.5 and a - 0.5 for a = 0.636;
    a for a = 0.202 in row 0), and moving up by s crosses the top wall over
    s from the last row only."""
    lat = orc.OracleLattice(4, 3)
    g = orc.OracleGrid(lat, 1, 4, tau=1.0, dy=DY4, collide=False, walls=True)
    for l in range(lat.q):
        s = lat.s[l, 1]
        for j in range(4):
            f = np.zeros((lat.q, 4, 1))
            f[l, j, 0] = 1.0
            lo, hi = g.wall_incident(f)
            e0, e1 = np.concatenate([[0.0], np.cumsum(DY4)])[[j, j + 1]]
            want_lo = max(0.0, min(e1 + s, 0.0) - (e0 + s)) if s < 0 else 0.0
            want_hi = max(0.0, (e1 + s) - max(e0 + s, 3.0)) if s > 0 else 0.0
            assert abs(lo[0] - want_lo) < 1e-15 and abs(hi[0] - want_hi) < 1e-15, (l, j)
    # explicit values for the outer and inner downward displacements
    l_out = next(l for l in range(lat.q) if lat.s[l, 1] < -0.6)
    l_in = next(l for l in range(lat.q) if -0.3 < lat.s[l, 1] < 0)
    a_out, a_in = -lat.s[l_out, 1], -lat.s[l_in, 1]
    for l, j, want in ((l_out, 0, 0.5), (l_out, 1, a_out - 0.5), (l_out, 2, 0.0),
                       (l_in, 0, a_in), (l_in, 1, 0.0)):
        f = np.zeros((lat.q, 4, 1))
        f[l, j, 0] = 1.0
        assert abs(g.wall_incident(f)[0][0] - want) < 1e-15, (l, j)


def test_two_height_rows_emission_interval(orc):
    """The bottom wall emits an upward population of displacement s into
    [0, s]: with rows (0.5, 0.5, ...) and s = 0.636 the first row is filled
    (overlap 0.5 over dy 0.5) and the second receives (s - 0.5)/0.5 of the
    same ghost value; for s = 0.202 only the first row, at s/0.5."""
    lat = orc.OracleLattice(4, 3)
    g = orc.OracleGrid(lat, 1, 4, tau=1.0, dy=DY4, collide=False, walls=True,
                       wall_lo=(0.0, 1.0), wall_hi=(0.0, 1.0))
    l_down = next(l for l in range(lat.q) if lat.s[l, 1] < -0.6)
    f = np.zeros((lat.q, 4, 1))
    f[l_down, 0, 0] = 1.0  # incident mass 0.5 through the bottom wall
    out = g.stream(f)
    outer = [l for l in range(lat.q) if lat.s[l, 1] > 0.6]
    inner = [l for l in range(lat.q) if 0 < lat.s[l, 1] < 0.3]
    for l in outer:
        s = lat.s[l, 1]
        ghost = out[l, 0, 0]
        assert ghost > 0
        assert abs(out[l, 1, 0] - ghost * (s - 0.5) / 0.5) < 1e-15
        assert np.all(out[l, 2:, 0] == 0)
    for l in inner:
        assert out[l, 0, 0] > 0 and np.all(out[l, 1:, 0] == 0)
    # the emitted ghost values of the outer and inner sets are in the ratio
    # of their wall equilibria: inner row 0 holds (s_in / 0.5) g_in
    for lo, li in zip(outer, inner):
        ratio = (out[lo, 0, 0]) / (out[li, 0, 0] / (lat.s[li, 1] / 0.5))
        assert abs(ratio - g.g.fw_lo[lo] / g.g.fw_lo[li]) < 1e-13


# ----------------------------------------------------------------- totals --
@pytest.mark.parametrize("n,order", [(4, 3), (6, 4)])
def test_totals_of_row_equilibria_closed_form(orc, n, order):
    """Each row j at its own equilibrium (rho_j, u_j, v_j, T_j) on rows of
    different heights: M = sum rho A, P = sum rho u A, E = sum (rho T +
    rho |u|^2 / 2) A with A = n_x dy_j (Sec. II with D = 2)."""
    lat = orc.OracleLattice(n, order)
    dy = np.array([0.5, 0.5, 1.0, 1.0, 0.25, 0.75, 1.0])
    nx, ny = 5, len(dy)
    g = orc.OracleGrid(lat, nx, ny, tau=1.0, dy=dy)
    rng = np.random.default_rng(12)
    rho = 1 + 0.2 * rng.random(ny)
    u = 0.1 * rng.standard_normal(ny)
    v = 0.1 * rng.standard_normal(ny)
    T = 1 + 0.1 * rng.standard_normal(ny)
    f = g.set_fields(*[np.repeat(a[:, None], nx, axis=1) for a in (rho, u, v, T)])
    A = nx * dy
    want = np.array([np.sum(rho * A), np.sum(rho * u * A), np.sum(rho * v * A),
                     np.sum((rho * T + 0.5 * rho * (u * u + v * v)) * A)])
    np.testing.assert_allclose(g.totals(f), want, rtol=1e-14, atol=1e-14 * want[0])


# ------------------------------------------------- mini-oracle agreement --
CASES = [
    dict(n=4, order=3, nx=5, dy=np.ones(4), tau=0.8, walls=False, steps=20),
    dict(n=6, order=4, nx=4, dy=np.ones(5), tau=0.6, walls=False, steps=12),
    dict(n=3, order=2, nx=5, dy=np.ones(4), tau=0.9, walls=False, steps=10, cfl=1.0, euclid=False),
    dict(n=4, order=3, nx=4, dy=np.ones(6), tau=0.7, walls=True, steps=20),
    dict(n=4, order=3, nx=3, dy=np.array([0.5, 0.5, 1, 1, 1, 0.5, 0.5]), tau=0.7, walls=True,
         steps=20),
    dict(n=6, order=4, nx=3, dy=np.array([0.25, 0.25, 0.5, 1, 1, 0.5, 0.25, 0.25]), tau=0.9,
         walls=True, steps=8),
    dict(n=4, order=3, nx=4, dy=np.array([0.5, 1.0, 0.25, 0.25, 1.0]), tau=0.75, walls=False,
         steps=15),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_mini_oracle_agrees_with_c_oracle(orc, case):
    c = CASES[case]
    cfl, euclid = c.get("cfl", 0.9), c.get("euclid", True)
    lat = orc.OracleLattice(c["n"], c["order"], cfl=cfl, cfl_norm=0 if euclid else 1)
    ml = mini.MiniLattice(c["n"], c["order"], cfl=cfl, euclid=euclid)
    np.testing.assert_allclose(ml.xi, lat.xi, atol=1e-14)
    np.testing.assert_allclose(ml.w, lat.w, rtol=1e-13)
    np.testing.assert_allclose(ml.s, lat.s, atol=1e-15)
    nx, dy = c["nx"], c["dy"]
    ny = len(dy)
    walls = dict(walls=c["walls"], wall_lo=(0.0, 1.0), wall_hi=(0.04, 1.08))
    g = orc.OracleGrid(lat, nx, ny, tau=c["tau"], dy=dy, **walls)
    mg = mini.MiniGrid(ml, nx, dy, tau=c["tau"], **walls)
    fields = inputs.shear_wave_fields(nx, ny, eps=0.03)
    noise = inputs.population_noise(lat.q, ny, nx, amp=1e-3, seed=case)
    f_c = g.set_fields(*fields, noise)
    f_m = mg.set_fields(*fields, noise)
    np.testing.assert_allclose(f_m, f_c, atol=2e-15)
    tc = g.totals(f_c)
    np.testing.assert_allclose(mg.totals(f_m), tc, rtol=1e-14, atol=1e-14 * tc[0])
    for _ in range(c["steps"]):
        f_c = g.step(f_c)
        f_m = mg.step(f_m)
    scale = np.max(np.abs(f_c))
    assert np.max(np.abs(f_m - f_c)) <= 1e-13 * scale
    tc = g.totals(f_c)
    np.testing.assert_allclose(mg.totals(f_m), tc, rtol=1e-13, atol=1e-13 * tc[0])
