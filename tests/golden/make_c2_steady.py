"""Write c2_steady_oracle.txt: the FP64 oracle's steady state of the bounded
thermal flow (Sec. VII diffuse walls, Sec. III rows refined 2:1 in 16-cell
bands at each wall: 288 rows, H = 256), D2Q16, tau 0.7, bottom wall at rest
with T = 1, top wall u = 0.05, T = 1.1, from the uniform state rho = 1, u = 0,
T = 1, stepped until the residual r = ||q^n - q^{n-K}|| / (K ||q^n||) over
K = 100 steps of the stacked fields q = (rho, u_x, u_y, T) falls below 1e-8.

The flow is invariant in x (periodic, uniform start, x-independent walls),
and every column of the oracle does the same arithmetic, so one column
gives the state of every column of the 512-column channel bitwise.

Calls only the oracle and the seeded input generators.  Run from the
repository root:  OMP_NUM_THREADS=1 python tests/golden/make_c2_steady.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_1004_5059_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_steady_oracle.txt")
K, TOL = 100, 1e-8


def main():
    dy = inputs.refined_wall_rows(h=256, band=16, ratio=2)
    ny = len(dy)
    lat = orc.OracleLattice(4, 3)
    g = orc.OracleGrid(lat, 1, ny, tau=0.7, dy=dy, walls=True, wall_lo=(0.0, 1.0),
                       wall_hi=(0.05, 1.1))
    f = g.set_fields(*inputs.uniform_fields(1, ny))
    m0 = g.totals(f)[0]
    q_prev = g.fields(f)
    steps, r = 0, np.inf
    while r >= TOL and steps < 2_000_000:
        f = g.run(f, K)
        steps += K
        q = g.fields(f)
        r = orc.residual(q, q_prev, K)
        q_prev = q
        if steps % 20000 == 0:
            print(f"step {steps}: r = {r:.3e}", flush=True)
    q = g.fields(f)[:, :, 0]
    drift = (g.totals(f)[0] - m0) / m0
    with open(OUT, "w") as fh:
        fh.write("# FP64 oracle steady state of the bounded thermal flow: D2Q16 (order 3), tau 0.7,\n")
        fh.write("# rows refined 2:1 in 16-cell bands at both walls (288 rows, H = 256), walls\n")
        fh.write("# (u, T) = (0, 1) at y = 0 and (0.05, 1.1) at y = H, uniform start, stepped until\n")
        fh.write(f"# the K = {K} residual is below {TOL:g}.  Written by make_c2_steady.py (oracle only).\n")
        fh.write(f"# steps {steps} residual {r:.17g} mass_drift {drift:.17g}\n")
        fh.write("# row dy rho ux uy T\n")
        for j in range(ny):
            fh.write(f"{j} {dy[j]:.17g} {q[0, j]:.17g} {q[1, j]:.17g} {q[2, j]:.17g} {q[3, j]:.17g}\n")
    print(f"wrote {OUT}: {steps} steps, r = {r:.3e}, mass drift {drift:.3e}")


if __name__ == "__main__":
    main()
