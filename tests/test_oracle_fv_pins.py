"""Pins of the finite-volume oracle (eq.(FVLB), eq.(FVLB2), eq.(IMPOSITION)):
each check rests on something other than the oracle's own code -- the
closed-form Fourier symbol of the stencils, the linearised Maxwellian, the
collision invariants, the flux balance of the re-emission, and the mesh
spacings the paper prints."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1004_5059_amd import inputs


@pytest.fixture(scope="module")
def lat():
    return orc.OracleLattice(4, 3)


def _mode(nx, ny, dx, dy, kx, ky):
    x = np.arange(nx) * dx
    y = np.arange(ny) * dy
    return kx * x[None, :] + ky * y[:, None]


@pytest.mark.parametrize("dx,dy,mx,my", [(1.0, 1.0, 1, 2), (0.5, 0.25, 3, 1), (1.0, 2.0, 5, 4)])
def test_streaming_symbol_is_the_stencils_closed_form(lat, dx, dy, mx, my):
    """Collision off: f_l = cos(theta) goes to cos(theta) + dt (c_x s_x +
    c_y s_y) sin(theta) with s_x = sin(kx dx)/dx (3/4 + cos(ky dy)/4) and
    s_y likewise: the 9-point stencils are central differences averaged
    3:1:... across the other axis."""
    nx, ny, dt = 24, 16, 0.05
    kx, ky = 2 * np.pi * mx / (nx * dx), 2 * np.pi * my / (ny * dy)
    th = _mode(nx, ny, dx, dy, kx, ky)
    g = orc.OracleFVGrid(lat, nx, ny, dx=dx, dt=dt, tau=1.0, dy=np.full(ny, dy), collide=False)
    f = np.repeat(np.cos(th)[None], lat.q, axis=0)
    out = g.step(f)
    sx = np.sin(kx * dx) / dx * (0.75 + 0.25 * np.cos(ky * dy))
    sy = np.sin(ky * dy) / dy * (0.75 + 0.25 * np.cos(kx * dx))
    for l in range(lat.q):
        cx, cy = lat.xi[l]
        expect = np.cos(th) + dt * (cx * sx + cy * sy) * np.sin(th)
        assert np.max(np.abs(out[l] - expect)) <= 1e-13


def test_linearised_step_matches_the_hermite_jacobian(lat):
    """Near rest the step is linear: for a Fourier mode,
    df' = df + dt [ -sigma_O (I - J)/tau df - (c.grad) df ] with
    J_lm = w_l [1 + xi_l.xi_m + (c_l^2 - D)(c_m^2 - D)/(2D)] (the
    Maxwellian's first-order Hermite terms) and the collision stencil's
    symbol sigma_O = (3/4 + cos kx/4)(3/4 + cos ky/4)."""
    nx, ny, dx, dt, tau = 16, 12, 1.0, 0.1, 0.7
    kx, ky = 2 * np.pi * 2 / nx, 2 * np.pi * 1 / ny
    th = _mode(nx, ny, dx, dx, kx, ky)
    rng = np.random.default_rng(3)
    amp = 1e-7 * rng.standard_normal(lat.q)
    w = lat.w
    c2 = (lat.xi ** 2).sum(axis=1)
    J = w[:, None] * (1.0 + lat.xi @ lat.xi.T + np.outer(c2 - 2, c2 - 2) / 4.0)
    g = orc.OracleFVGrid(lat, nx, ny, dx=dx, dt=dt, tau=tau)
    f = w[:, None, None] + amp[:, None, None] * np.cos(th)[None]
    out = g.step(f) - w[:, None, None]
    sig_o = (0.75 + 0.25 * np.cos(kx)) * (0.75 + 0.25 * np.cos(ky))
    sx = np.sin(kx) * (0.75 + 0.25 * np.cos(ky))
    sy = np.sin(ky) * (0.75 + 0.25 * np.cos(kx))
    a_cos = amp - dt * sig_o * ((np.eye(lat.q) - J) @ amp) / tau
    a_sin = dt * (lat.xi[:, 0] * sx + lat.xi[:, 1] * sy) * amp
    expect = a_cos[:, None, None] * np.cos(th)[None] + a_sin[:, None, None] * np.sin(th)[None]
    assert np.max(np.abs(out - expect)) <= 1e-6 * np.max(np.abs(amp))


def test_conservation_on_a_nonuniform_periodic_mesh(lat):
    """Mass, momentum and energy with the dual-cell weights dx (dy_{j-1} +
    dy_j)/2: the flux stencils telescope and the collision term's
    invariants vanish at every point."""
    nx, ny = 20, 18
    rng = np.random.default_rng(1)
    dy = rng.uniform(0.4, 1.6, ny)
    g = orc.OracleFVGrid(lat, nx, ny, dx=0.8, dt=0.05, tau=0.6, dy=dy)
    y = np.cumsum(dy) / dy.sum()
    f = g.set_fields(1 + 0.01 * np.cos(2 * np.pi * y)[:, None] * np.ones((1, nx)),
                     0.02 * np.sin(2 * np.pi * y)[:, None] * np.ones((1, nx)), 0.01,
                     1 + 0.03 * np.cos(4 * np.pi * y)[:, None] * np.ones((1, nx)),
                     inputs.population_noise(lat.q, ny, nx, amp=1e-4, seed=2))
    t0 = g.totals(f)
    t1 = g.totals(g.run(f, 200))
    assert abs(t1[0] - t0[0]) / t0[0] <= 1e-13
    assert np.max(np.abs(t1[1:3] - t0[1:3])) / t0[0] <= 1e-13
    assert abs(t1[3] - t0[3]) / t0[3] <= 1e-13


def test_uniform_equilibrium_is_a_fixed_point(lat):
    g = orc.OracleFVGrid(lat, 10, 9, dx=1.0, dt=0.1, tau=0.8,
                         dy=np.linspace(0.5, 1.5, 9))
    f = g.set_fields(1.0, 0.03, -0.02, 1.05)
    assert np.max(np.abs(g.run(f, 20) - f)) <= 1e-15


def test_wall_re_emission_balances_the_normal_flux(lat):
    """eq.(IMPOSITION): after re-emission the net normal mass flux of every
    wall point is zero, and its outgoing populations are proportional to
    the wall Maxwellian."""
    nx, ny = 12, 10
    g = orc.OracleFVGrid(lat, nx, ny, dx=1.0, dt=0.1, tau=0.8, walls=True,
                         wall_lo=(0.0, 1.0), wall_hi=(0.05, 1.1))
    rng = np.random.default_rng(4)
    f = lat.w[:, None, None] * (1 + 0.05 * rng.standard_normal((lat.q, ny, nx)))
    fi = g.impose(f)
    cy = lat.xi[:, 1]
    for j, (uw, Tw), sgn in ((0, (0.0, 1.0), 1), (ny - 1, (0.05, 1.1), -1)):
        flux = np.einsum("l,li->i", cy, fi[:, j, :])
        assert np.max(np.abs(flux)) <= 1e-15
        out = sgn * cy > 0
        feq = lat.feq(1.0, uw, 0.0, Tw)
        ratio = fi[out, j, :] / feq[out][:, None]
        assert np.max(np.abs(ratio - ratio[0])) <= 1e-14
        assert np.array_equal(fi[~out, j, :], f[~out, j, :])


def test_rest_state_between_resting_walls_is_a_fixed_point(lat):
    ny = 9
    g = orc.OracleFVGrid(lat, 8, ny, dx=1.0, dt=0.1, tau=0.8, walls=True,
                         dy=np.linspace(0.5, 1.0, ny - 1))
    f = g.set_fields(1.0, 0.0, 0.0, 1.0)
    assert np.max(np.abs(g.run(f, 30) - f)) <= 1e-15


def test_tanh_mesh_spacings_are_the_papers():
    """Sec. X: beta = 2.3, N_y = 60, L_y = 10 gives spacings from
    0.016631 at the walls to 0.391 in the middle (60 equal steps of phi)."""
    y = inputs.tanh_mesh(10.0, 60, 2.3)
    d = np.diff(y)
    assert len(y) == 61 and y[0] == 0.0 and abs(y[-1] - 10.0) < 1e-12
    assert abs(d.min() - 0.016631) < 2e-6
    assert abs(d.max() - 0.391) < 1e-3
    assert np.allclose(d, d[::-1], rtol=1e-12)
