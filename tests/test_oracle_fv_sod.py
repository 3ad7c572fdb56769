"""Pins of the oracle for the compressible workload of Sec. VI: the
fifth-order equilibrium of Appendix A on the 6-point Gauss-Hermite set
(D2Q36), the zero-gradient (adiabatic) x ends, and the Sod shock tube
against the exact Riemann solution of the inviscid Euler equations for the
two-dimensional ideal gas of the model (gamma = c_P / c_v = 2)."""
import math

import numpy as np
import pytest

import sod_exact as se
from oracle import oracle as orc

LEFT, RIGHT, GAMMA = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 2.0


def _gauss_moment(mu, var, k):
    """E[(mu + sqrt(var) Z)^k], Z standard normal (binomial expansion)."""
    return sum(math.comb(k, i) * mu ** (k - i) * (var ** (i // 2) * _dfact(i - 1) if i % 2 == 0 else 0.0)
               for i in range(k + 1))


def _dfact(n):
    return 1 if n <= 0 else n * _dfact(n - 2)


def test_fifth_order_equilibrium_carries_the_maxwellian_moments():
    """sum_l feq x^i y^j = rho E[X^i] E[Y^j] for the Maxwellian (independent
    Gaussians of means u_x, u_y and variance T) for every i + j <= 5 on
    D2Q36 with the order-5 equilibrium; order 4 misses the fifth moments."""
    rng = np.random.default_rng(11)
    for order, top in ((5, 5), (4, 4)):
        lat = orc.OracleLattice(6, order)
        for _ in range(4):
            rho, ux, uy, T = 1 + 0.3 * rng.random(), 0.4 * rng.standard_normal(), \
                0.4 * rng.standard_normal(), 0.7 + 0.6 * rng.random()
            feq = lat.feq(rho, ux, uy, T)
            for i in range(6):
                for j in range(6 - i):
                    got = np.sum(feq * lat.xi[:, 0] ** i * lat.xi[:, 1] ** j)
                    want = rho * _gauss_moment(ux, T, i) * _gauss_moment(uy, T, j)
                    if i + j <= top:
                        assert abs(got - want) <= 1e-11 * max(1.0, abs(want))
        if order == 4:  # some fifth moment differs
            assert abs(np.sum(feq * lat.xi[:, 0] ** 5) - rho * _gauss_moment(ux, T, 5)) > 1e-6


def test_zero_gradient_ends_keep_a_uniform_state():
    lat = orc.OracleLattice(6, 5)
    g = orc.OracleFVGrid(lat, 30, 4, dx=0.1, dt=0.01, tau=0.05, dy=np.full(4, 0.1), x_open=True)
    f = g.set_fields(1.1, 0.0, 0.0, 0.9)
    assert np.max(np.abs(g.run(f, 50) - f)) <= 1e-15


def _sod(order, nx=200, tau=0.001, dt=2e-4, t_end=0.1):
    lat = orc.OracleLattice(6, order)
    dx = 1.0 / nx
    g = orc.OracleFVGrid(lat, nx, 2, dx=dx, dt=dt, tau=tau, dy=np.full(2, dx), x_open=True)
    x = np.arange(nx) * dx
    h = 0.5 * (1 - np.tanh((x - 0.5) / 0.007))  # Sec. VI: tanh step of width 0.007
    rho, p = 0.125 + 0.875 * h, 0.1 + 0.9 * h
    r2 = np.tile(rho, (2, 1))
    f = g.set_fields(r2, 0 * r2, 0 * r2, np.tile(p / rho, (2, 1)))
    t0 = g.totals(f)
    f = g.run(f, int(round(t_end / dt)))
    return x, g.fields(f), t0, g.totals(f)


def test_sod_tube_follows_the_riemann_solution():
    """tau = 0.001 (the inviscid limit is approached as tau -> 0; Sec. VI uses
    0.005 at a finer mesh), 200 points, t = 0.1: the star pressure and the
    velocity behind the rarefaction within 1 %, the density within L1 0.012,
    the shock within two points; mass and energy conserved (no wave reaches
    the ends), x momentum changed by the end pressures, (p_L - p_R) L_y t."""
    x, F, t0, t1 = _sod(5)
    ex = se.sample(x, 0.1, 0.5, LEFT, RIGHT, GAMMA)
    ps, us = se.star_state(LEFT, RIGHT, GAMMA)
    star = np.where(np.abs(ex[1] - us) < 1e-12)[0]
    left = star[2:len(star) // 3]
    assert abs(np.mean(F[1][0][left]) / us - 1) <= 0.01
    assert abs(np.mean((F[0][0] * F[3][0])[star]) / ps - 1) <= 0.01
    assert np.mean(np.abs(F[0][0] - ex[0])) <= 0.012
    half = 0.5 * (ex[0][star[-1]] + RIGHT[0])
    assert abs(x[np.where(F[0][0] > half)[0].max()] - x[np.where(ex[0] > half)[0].max()]) <= 2.01 / 200
    assert abs(t1[0] - t0[0]) / t0[0] <= 1e-12 and abs(t1[3] - t0[3]) / t0[3] <= 1e-12
    ly = 2.0 / 200
    assert abs(t1[1] - (LEFT[2] - RIGHT[2]) * ly * 0.1) <= 0.02 * (LEFT[2] - RIGHT[2]) * ly * 0.1


@pytest.mark.parametrize("n,order", [(4, 3), (6, 4), (6, 5)])
def test_zero_gradient_ends_exchange_only_the_end_fluxes(n, order):
    """With the end point standing in for its missing x neighbour, the
    central x differences of eq.(FVLB) telescope over the row to the two end
    points, and the x smoothing of the collision term sums to one.  On a
    uniform periodic y mesh each collision invariant phi (1, c_x, c_y,
    |c|^2 / 2) therefore changes per step by exactly
    -dt dy sum_j sum_l phi_l c_x (f_l(x_end, y_j) - f_l(x_0, y_j)),
    whatever the state: the conservation law the Sod pins rely on while no
    population has reached the ends."""
    lat = orc.OracleLattice(n, order)
    nx, ny, dx, dt = 40, 4, 0.1, 0.004
    g = orc.OracleFVGrid(lat, nx, ny, dx=dx, dt=dt, tau=0.05, dy=np.full(ny, dx), x_open=True)
    X, Y = np.meshgrid(np.arange(nx) * dx, np.arange(ny) * dx)
    f = g.set_fields(1 + 0.2 * np.sin(1.3 * X) + 0.05 * np.cos(2 * np.pi * Y / (ny * dx)),
                     0.1 + 0.05 * np.cos(0.7 * X), 0.02 + 0.03 * np.sin(2 * np.pi * Y / (ny * dx)),
                     1 + 0.1 * np.cos(0.9 * X + 0.4))
    cx, cy = lat.xi[:, 0], lat.xi[:, 1]
    phi = np.stack([np.ones_like(cx), cx, cy, 0.5 * (cx * cx + cy * cy)])
    for _ in range(3):
        t0 = g.totals(f)
        jump = np.sum(f[:, :, -1] - f[:, :, 0], axis=1)  # sum over y, per population
        want = -dt * dx * (phi * cx) @ jump
        f = g.step(f)
        got = g.totals(f) - t0
        assert np.all(np.abs(want) > 1e-6)  # the ends do exchange every invariant here
        assert np.allclose(got, want, rtol=1e-10, atol=1e-14 * np.abs(t0).max())
