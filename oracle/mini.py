"""NumPy mini-oracle of the TVLBM step, for tiny grids.

TEST INFRASTRUCTURE ONLY: imported by tests/ to cross-check the C oracle
(tvlbm_oracle.c).  It shares no code with the C oracle or with the HIP
library, and the product package never imports it.

It restates the same definitions with a different construction, so that a
slip in either implementation shows up as a disagreement:

* velocity set: numpy's Gauss-Hermite rule (hermegauss) instead of the
  Golub-Welsch eigenproblem;
* equilibrium (Sec. II, Appendix A): the Hermite expansion of the
  Maxwellian built from the closed-form 1-D coefficients
  a_p(u, T) = E[He_p(X)], X ~ N(u, T), i.e.
  a_p = sum_k p! / (k! (p - 2k)!) u^(p-2k) ((T - 1)/2)^k, multiplied over the
  two axes and truncated at total order N, instead of the scalar form of
  Appendix A;
* moments (Sec. II): rho, rho u and the central second moment, vectorised;
* collision: f* = f - (f - feq)/tau, tau in steps;
* volumetric streaming: each population moved by the dense matrices of the
  exact-overlap remap along x (unit cells) and y (rows of heights dy), the
  y matrix built from interval intersections of the shifted source rows
  with the target rows (periodic images, or walls);
* diffuse walls: the mass carried through a wall by the shifted cells of the
  incident populations, per landing column, is re-emitted into the outgoing
  populations in proportion to displacement-weighted wall equilibria (the
  flux-weighted ratio of eq.(IMPOSITION), |c.n| dt = displacement), placed
  in the interval between the wall and the displaced wall.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import hermite_e as He


class MiniLattice:
    def __init__(self, n: int, order: int, cfl: float = 0.9, euclid: bool = True):
        x, w = He.hermegauss(n)
        x = 0.5 * (x - x[::-1])  # exact symmetry about 0
        w = 0.5 * (w + w[::-1]) / math.sqrt(2.0 * math.pi)
        self.n, self.q, self.order = n, n * n, order
        self.x1, self.w1 = x, w
        a, b = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        self.xi = np.stack([x[a.ravel()], x[b.ravel()]], axis=1)  # l = a n + b
        self.w = (w[a.ravel()] * w[b.ravel()])
        cmax = math.sqrt(2.0) * x.max() if euclid else x.max()
        self.lam = cfl / cmax
        s = self.lam * self.xi
        r = np.rint(s)
        self.s = np.where(np.abs(s - r) <= 4 * np.spacing(np.abs(s)), r, s)

    @staticmethod
    def _coef(p: int, u: float, T: float) -> float:
        h = 0.5 * (T - 1.0)
        return sum(math.factorial(p) / (math.factorial(k) * math.factorial(p - 2 * k))
                   * u ** (p - 2 * k) * h ** k for k in range(p // 2 + 1))

    def feq(self, rho: float, ux: float, uy: float, T: float) -> np.ndarray:
        out = np.zeros(self.q)
        for p in range(self.order + 1):
            cp = np.zeros(p + 1)
            cp[p] = 1.0
            hx = He.hermeval(self.xi[:, 0], cp) * self._coef(p, ux, T) / math.factorial(p)
            for q in range(self.order + 1 - p):
                cq = np.zeros(q + 1)
                cq[q] = 1.0
                hy = He.hermeval(self.xi[:, 1], cq) * self._coef(q, uy, T) / math.factorial(q)
                out += hx * hy
        return self.w * rho * out

    def moments(self, f: np.ndarray):
        """f [q][...] -> rho, ux, uy, T arrays."""
        rho = f.sum(axis=0)
        ux = np.tensordot(self.xi[:, 0], f, axes=1) / rho
        uy = np.tensordot(self.xi[:, 1], f, axes=1) / rho
        cx = self.xi[:, 0].reshape((-1,) + (1,) * (f.ndim - 1)) - ux
        cy = self.xi[:, 1].reshape((-1,) + (1,) * (f.ndim - 1)) - uy
        T = ((cx * cx + cy * cy) * f).sum(axis=0) / (2.0 * rho)
        return rho, ux, uy, T


def _shift_matrix_unit(n: int, s: float) -> np.ndarray:
    """Periodic remap of n unit cells displaced by s (|s| <= 1):
    M[target, source]; source i moves to [i + s, i + 1 + s]."""
    m = math.floor(s)
    phi = s - m
    M = np.zeros((n, n))
    for i in range(n):
        M[(i + m) % n, i] += 1.0 - phi
        M[(i + m + 1) % n, i] += phi
    return M


def _ov(a0, a1, b0, b1):
    return max(0.0, min(a1, b1) - max(a0, b0))


class MiniGrid:
    """Grid of nx unit columns and rows of heights dy (periodic or walled)."""

    def __init__(self, lat: MiniLattice, nx: int, dy, tau: float, walls: bool = False,
                 wall_lo=(0.0, 1.0), wall_hi=(0.0, 1.0), collide: bool = True):
        self.lat, self.nx = lat, nx
        self.dy = np.asarray(dy, dtype=np.float64)
        self.ny = len(self.dy)
        self.tau, self.walls, self.do_collide = tau, walls, collide
        edges = np.concatenate([[0.0], np.cumsum(self.dy)])
        self.H = edges[-1]
        self.Sx, self.Sy, self.Gy, self.Iy = [], [], [], []
        for l in range(lat.q):
            sx, sy = lat.s[l]
            self.Sx.append(_shift_matrix_unit(nx, sx))
            Sy = np.zeros((self.ny, self.ny))
            G = np.zeros(self.ny)   # ghost interval overlap / dy_k
            I = np.zeros(self.ny)   # length of shifted source row j beyond a wall
            for j in range(self.ny):
                a0, a1 = edges[j] + sy, edges[j + 1] + sy
                for k in range(self.ny):
                    b0, b1 = edges[k], edges[k + 1]
                    L = _ov(a0, a1, b0, b1)
                    if not walls:
                        L += _ov(a0 - self.H, a1 - self.H, b0, b1) + _ov(a0 + self.H, a1 + self.H, b0, b1)
                    Sy[k, j] = L / self.dy[k]
                if walls:
                    I[j] = _ov(a0, a1, -np.inf, 0.0) + _ov(a0, a1, self.H, np.inf)
            if walls:
                for k in range(self.ny):
                    b0, b1 = edges[k], edges[k + 1]
                    G[k] = (_ov(0.0, sy, b0, b1) if sy > 0 else _ov(self.H + sy, self.H, b0, b1)) / self.dy[k]
            self.Sy.append(Sy)
            self.Gy.append(G)
            self.Iy.append(I)
        if walls:
            self.fw_lo = lat.feq(1.0, wall_lo[0], 0.0, wall_lo[1])
            self.fw_hi = lat.feq(1.0, wall_hi[0], 0.0, wall_hi[1])

    def set_fields(self, rho, ux, uy, T, noise=None) -> np.ndarray:
        f = np.zeros((self.lat.q, self.ny, self.nx))
        b = [np.broadcast_to(a, (self.ny, self.nx)) for a in (rho, ux, uy, T)]
        for j in range(self.ny):
            for i in range(self.nx):
                f[:, j, i] = self.lat.feq(b[0][j, i], b[1][j, i], b[2][j, i], b[3][j, i])
        return f if noise is None else f + noise

    def collide(self, f):
        if not self.do_collide:
            return f.copy()
        rho, ux, uy, T = self.lat.moments(f)
        out = np.empty_like(f)
        for j in range(self.ny):
            for i in range(self.nx):
                fe = self.lat.feq(rho[j, i], ux[j, i], uy[j, i], T[j, i])
                out[:, j, i] = f[:, j, i] - (f[:, j, i] - fe) / self.tau
        return out

    def stream(self, fs):
        lat = self.lat
        out = np.zeros_like(fs)
        xs = [fs[l] @ self.Sx[l].T for l in range(lat.q)]  # x remap of every row
        if self.walls:
            m_lo = np.zeros(self.nx)
            m_hi = np.zeros(self.nx)
            for l in range(lat.q):
                sy = lat.s[l, 1]
                inc = self.Iy[l] @ xs[l]  # per landing column
                if sy < 0:
                    m_lo += inc
                elif sy > 0:
                    m_hi += inc
            z_lo = sum(lat.s[l, 1] * self.fw_lo[l] for l in range(lat.q) if lat.s[l, 1] > 0)
            z_hi = sum(-lat.s[l, 1] * self.fw_hi[l] for l in range(lat.q) if lat.s[l, 1] < 0)
        for l in range(lat.q):
            o = self.Sy[l] @ xs[l]
            if self.walls:
                sy = lat.s[l, 1]
                if sy > 0:
                    ghost = (m_lo * self.fw_lo[l] / z_lo) @ self.Sx[l].T
                elif sy < 0:
                    ghost = (m_hi * self.fw_hi[l] / z_hi) @ self.Sx[l].T
                else:
                    ghost = np.zeros(self.nx)
                o = o + np.outer(self.Gy[l], ghost)
            out[l] = o
        return out

    def step(self, f):
        return self.stream(self.collide(f))

    def run(self, f, n: int):
        for _ in range(n):
            f = self.step(f)
        return f

    def totals(self, f):
        """M, Px, Py, E with E = 1/2 sum |xi|^2 f, weighted by cell areas."""
        lat = self.lat
        a = f * self.dy[None, :, None]
        c2 = (lat.xi ** 2).sum(axis=1)
        return np.array([a.sum(), np.tensordot(lat.xi[:, 0], a, axes=1).sum(),
                         np.tensordot(lat.xi[:, 1], a, axes=1).sum(),
                         0.5 * np.tensordot(c2, a, axes=1).sum()])
