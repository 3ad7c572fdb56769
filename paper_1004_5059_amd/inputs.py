"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds none of the method's arithmetic: it only draws numbers and
shapes them into initial macroscopic fields, population noise and instance
parameters.  Both the HIP path and the oracle turn these into populations
with their own equilibrium code.

Recipes (all synthetic; the paper's workloads are synthetic too):

* ``shear_wave_fields`` -- the transverse shear wave of the transport
  coefficient experiment (Sec. V): rho = 1, T = 1, u_x = eps sin(2 pi y / L_y)
  with y the row index, u_y = 0.
* ``population_noise`` -- uniform noise in [-amp, amp) per population and
  cell from a counter-based splitmix64 generator keyed by
  (seed, l, j, i), so any sub-block can be regenerated independently.
* ``smoothed_density_fields`` -- rho = 1 + std * (periodic Gaussian-smoothed
  N(0,1), zero mean, unit variance), T = 1 + amp sin(2 pi x / N_x), u = 0.
* ``couette_instances`` -- thermal Couette instances with N_y drawn from
  {32, 48, ..., 256}, N_x = N_y / 2, tau ~ U(0.55, 1.2), top-wall u_x ~
  U(0, 0.08), wall temperature difference ~ U(0, 0.2).
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(counter: np.ndarray) -> np.ndarray:
    """splitmix64 output for each 64-bit counter value (Steele, Lea & Flood,
    2014): state = (counter + 1) * golden-ratio increment, then the
    xor-shift-multiply finaliser."""
    with np.errstate(over="ignore"):
        z = (counter.astype(np.uint64) + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform01(seed: int, shape) -> np.ndarray:
    """Counter-based uniforms in [0, 1): counter = seed * 2^40 + flat index."""
    n = int(np.prod(shape))
    ctr = np.arange(n, dtype=np.uint64) + np.uint64(seed) * np.uint64(1 << 40)
    bits = splitmix64(ctr) >> np.uint64(11)
    return (bits.astype(np.float64) * (1.0 / 9007199254740992.0)).reshape(shape)


def population_noise(q: int, ny: int, nx: int, amp: float = 1e-4, seed: int = 0) -> np.ndarray:
    """[q][ny][nx] float64 noise, uniform in [-amp, amp)."""
    return amp * (2.0 * uniform01(seed, (q, ny, nx)) - 1.0)


def shear_wave_fields(nx: int, ny: int, eps: float = 0.01):
    """(rho, ux, uy, T), each [ny][nx] float64."""
    j = np.arange(ny, dtype=np.float64)[:, None]
    ux = eps * np.sin(2.0 * np.pi * j / ny) * np.ones((1, nx))
    one = np.ones((ny, nx))
    return one.copy(), ux, np.zeros((ny, nx)), one.copy()


def smoothed_density_fields(nx: int, ny: int, std: float = 0.01, sigma: float = 4.0,
                            t_amp: float = 0.05, seed: int = 1):
    """(rho, ux, uy, T), each [ny][nx] float64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((ny, nx))
    ky = 2.0 * np.pi * np.fft.fftfreq(ny)[:, None]
    kx = 2.0 * np.pi * np.fft.fftfreq(nx)[None, :]
    filt = np.exp(-0.5 * sigma * sigma * (kx * kx + ky * ky))
    s = np.real(np.fft.ifft2(np.fft.fft2(g) * filt))
    s = (s - s.mean()) / s.std()
    rho = 1.0 + std * s
    i = np.arange(nx, dtype=np.float64)[None, :]
    T = (1.0 + t_amp * np.sin(2.0 * np.pi * i / nx)) * np.ones((ny, 1))
    z = np.zeros((ny, nx))
    return rho, z, z.copy(), T


def uniform_fields(nx: int, ny: int, rho: float = 1.0, T: float = 1.0):
    one = np.ones((ny, nx))
    return rho * one, 0.0 * one, 0.0 * one, T * one


def couette_instances(n: int, seed: int = 2026, sizes=None):
    """List of dicts: nx, ny, tau, u_top, T_bot, T_top (bottom wall at rest).
    sizes: the N_y values to draw from (default 32, 48, ..., 256)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.arange(32, 257, 16) if sizes is None else np.asarray(sizes)
    out = []
    for _ in range(n):
        ny = int(rng.choice(sizes))
        tau = float(rng.uniform(0.55, 1.2))
        u_top = float(rng.uniform(0.0, 0.08))
        dT = float(rng.uniform(0.0, 0.2))
        out.append(dict(nx=ny // 2, ny=ny, tau=tau, u_top=u_top, T_bot=1.0, T_top=1.0 + dT))
    return out


def refined_wall_rows(h: int = 256, band: int = 16, ratio: int = 2) -> np.ndarray:
    """Row heights of a channel of height h whose first and last ``band``
    coarse rows are split ``ratio``:1 in y."""
    fine = np.full(band * ratio, 1.0 / ratio)
    coarse = np.ones(h - 2 * band)
    return np.concatenate([fine, coarse, fine])


def tanh_mesh(length: float = 10.0, n_spacings: int = 60, beta: float = 2.3) -> np.ndarray:
    """Mesh-point coordinates (ascending, n_spacings + 1 points from 0 to
    length) of the hyperbolic-tangent stretching of Sec. X:
    y = (L/2)(1 + tanh(beta phi)/tanh(beta)), phi running from -1 to 1 in
    n_spacings equal steps (spacings smallest at both walls)."""
    phi = 1.0 - 2.0 * np.arange(n_spacings + 1) / n_spacings
    y = 0.5 * length * (1.0 + np.tanh(beta * phi) / np.tanh(beta))
    return np.sort(y)
