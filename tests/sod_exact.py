"""Exact solution of the Riemann problem of the inviscid Euler equations for
an ideal gas (the reference of the shock-tube runs of Sec. VI), written from
the standard construction (Toro, Riemann Solvers and Numerical Methods for
Fluid Dynamics, ch. 4): the star pressure is the root of
f_L(p) + f_R(p) + u_R - u_L = 0, with f_K the shock (p > p_K) or
rarefaction (p <= p_K) branch, solved by Newton's method; the solution is
then sampled along x/t.  Test infrastructure; independent of the oracle."""
import numpy as np


def _f(p, rho, pk, gamma):
    a = np.sqrt(gamma * pk / rho)
    if p > pk:
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        q = np.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (B + p))
    r = p / pk
    return (2.0 * a / (gamma - 1.0)) * (r ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0), \
        r ** (-(gamma + 1.0) / (2.0 * gamma)) / (rho * a)


def star_state(left, right, gamma):
    rl, ul, pl = left
    rr, ur, pr = right
    p = 0.5 * (pl + pr)
    for _ in range(100):
        fl, dl = _f(p, rl, pl, gamma)
        fr, dr = _f(p, rr, pr, gamma)
        dp = (fl + fr + ur - ul) / (dl + dr)
        p = max(p - dp, 1e-12)
        if abs(dp) < 1e-15 * p:
            break
    fl, _ = _f(p, rl, pl, gamma)
    fr, _ = _f(p, rr, pr, gamma)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(x, t, x0, left, right, gamma):
    """(rho, u, p) at positions x and time t > 0, discontinuity at x0."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, gamma)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    al, ar = np.sqrt(gamma * pl / rl), np.sqrt(gamma * pr / rr)
    out = np.zeros((3, len(x)))
    for k, xv in enumerate(np.asarray(x, dtype=float)):
        s = (xv - x0) / t
        if s <= us:  # left of the contact
            if ps > pl:  # left shock
                sl = ul - al * np.sqrt((gamma + 1) / (2 * gamma) * ps / pl + (gamma - 1) / (2 * gamma))
                out[:, k] = (rl, ul, pl) if s <= sl else (rl * (ps / pl + g1) / (g1 * ps / pl + 1), us, ps)
            else:  # left rarefaction
                asl = al * (ps / pl) ** ((gamma - 1) / (2 * gamma))
                if s <= ul - al:
                    out[:, k] = (rl, ul, pl)
                elif s >= us - asl:
                    out[:, k] = (rl * (ps / pl) ** (1 / gamma), us, ps)
                else:
                    c = 2 / (gamma + 1) + g1 / al * (ul - s)
                    out[:, k] = (rl * c ** (2 / (gamma - 1)), 2 / (gamma + 1) * (al + (gamma - 1) / 2 * ul + s),
                                 pl * c ** (2 * gamma / (gamma - 1)))
        else:  # right of the contact
            if ps > pr:  # right shock
                sr = ur + ar * np.sqrt((gamma + 1) / (2 * gamma) * ps / pr + (gamma - 1) / (2 * gamma))
                out[:, k] = (rr, ur, pr) if s >= sr else (rr * (ps / pr + g1) / (g1 * ps / pr + 1), us, ps)
            else:  # right rarefaction
                asr = ar * (ps / pr) ** ((gamma - 1) / (2 * gamma))
                if s >= ur + ar:
                    out[:, k] = (rr, ur, pr)
                elif s <= us + asr:
                    out[:, k] = (rr * (ps / pr) ** (1 / gamma), us, ps)
                else:
                    c = 2 / (gamma + 1) - g1 / ar * (ur - s)
                    out[:, k] = (rr * c ** (2 / (gamma - 1)), 2 / (gamma + 1) * (-ar + (gamma - 1) / 2 * ur + s),
                                 pr * c ** (2 * gamma / (gamma - 1)))
    return out
