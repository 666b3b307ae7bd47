"""Exact solution of the Riemann problem of the 1D Euler equations of an
ideal gas (test helper, no GPU): the star pressure from the sum of the two
wave functions (shock: Rankine-Hugoniot; rarefaction: isentropic
characteristic relation), root by bracketing, then the extreme wave speeds
and the self-similar solution sampled at x / t (the textbook construction,
written here from those relations)."""
import math

import numpy as np
from scipy.optimize import brentq


def wave_fn(p, rho, pk, c, g):
    """Velocity jump across the left / right wave as a function of the star
    pressure p (shock for p > pk, rarefaction otherwise)."""
    if p > pk:
        a = 2.0 / ((g + 1.0) * rho)
        b = (g - 1.0) / (g + 1.0) * pk
        return (p - pk) * math.sqrt(a / (p + b))
    return 2.0 * c / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)


def _pstar(rhoL, vL, pL, rhoR, vR, pR, g):
    """Star pressure; 0 when the two rarefactions open a vacuum."""
    cL, cR = math.sqrt(g * pL / rhoL), math.sqrt(g * pR / rhoR)
    f = lambda p: wave_fn(p, rhoL, pL, cL, g) + wave_fn(p, rhoR, pR, cR, g) + (vR - vL)
    if f(0.0) >= 0.0:
        return 0.0
    hi = max(pL, pR)
    while f(hi) < 0.0:
        hi *= 2.0
    return brentq(f, 0.0, hi, xtol=1e-300, rtol=4 * np.finfo(float).eps, maxiter=500)


def extreme_speeds(rhoL, vL, pL, rhoR, vR, pR, g):
    """Star pressure and the two extreme wave speeds (S_left, S_right)."""
    cL, cR = math.sqrt(g * pL / rhoL), math.sqrt(g * pR / rhoR)
    ps = _pstar(rhoL, vL, pL, rhoR, vR, pR, g)
    if ps == 0.0:
        return 0.0, vL - cL, vR + cR
    kap = (g + 1.0) / (2.0 * g)
    sL = vL - cL * (math.sqrt(1.0 + kap * (ps / pL - 1.0)) if ps > pL else 1.0)
    sR = vR + cR * (math.sqrt(1.0 + kap * (ps / pR - 1.0)) if ps > pR else 1.0)
    return ps, sL, sR


def star_state(left, right, g=1.4):
    """(p*, u*) of the primitive states left = (rho, u, p), right = (...)
    (no vacuum)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps = _pstar(rl, ul, pl, rr, ur, pr, g)
    if ps == 0.0:
        raise ValueError("the rarefactions open a vacuum")
    us = 0.5 * (ul + ur) + 0.5 * (wave_fn(ps, rr, pr, cr, g) - wave_fn(ps, rl, pl, cl, g))
    return ps, us


def sample(left, right, xi, g=1.4):
    """Primitive (rho, u, p) of the exact solution at the similarity
    coordinates xi = (x - x0) / t (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    ps, us = star_state(left, right, g)
    xi = np.asarray(xi, dtype=float)
    rho, u, p = np.empty_like(xi), np.empty_like(xi), np.empty_like(xi)
    g1, g2 = (g - 1.0) / (2.0 * g), (g + 1.0) / (2.0 * g)
    r6 = (g - 1.0) / (g + 1.0)
    for k, s in enumerate(xi):
        if s <= us:                               # left of the contact
            if ps > pl:                           # left shock
                sl = ul - cl * np.sqrt(g2 * ps / pl + g1)
                if s <= sl:
                    rho[k], u[k], p[k] = rl, ul, pl
                else:
                    rho[k] = rl * (ps / pl + r6) / (r6 * ps / pl + 1.0)
                    u[k], p[k] = us, ps
            else:                                 # left rarefaction
                head = ul - cl
                cs = cl * (ps / pl) ** g1
                tail = us - cs
                if s <= head:
                    rho[k], u[k], p[k] = rl, ul, pl
                elif s >= tail:
                    rho[k], u[k], p[k] = rl * (ps / pl) ** (1.0 / g), us, ps
                else:                             # inside the fan
                    c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - s))
                    u[k] = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + s)
                    rho[k] = rl * (c / cl) ** (2.0 / (g - 1.0))
                    p[k] = pl * (c / cl) ** (2.0 * g / (g - 1.0))
        else:                                     # right of the contact
            if ps > pr:                           # right shock
                sr = ur + cr * np.sqrt(g2 * ps / pr + g1)
                if s >= sr:
                    rho[k], u[k], p[k] = rr, ur, pr
                else:
                    rho[k] = rr * (ps / pr + r6) / (r6 * ps / pr + 1.0)
                    u[k], p[k] = us, ps
            else:                                 # right rarefaction
                head = ur + cr
                cs = cr * (ps / pr) ** g1
                tail = us + cs
                if s >= head:
                    rho[k], u[k], p[k] = rr, ur, pr
                elif s <= tail:
                    rho[k], u[k], p[k] = rr * (ps / pr) ** (1.0 / g), us, ps
                else:
                    c = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - s))
                    u[k] = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + s)
                    rho[k] = rr * (c / cr) ** (2.0 / (g - 1.0))
                    p[k] = pr * (c / cr) ** (2.0 * g / (g - 1.0))
    return rho, u, p


def cell_averages(left, right, x0, t, edges, g=1.4, nq=16):
    """Exact cell averages of the conserved variables (rho, rho u, E) over
    the cells [edges[i], edges[i+1]] -> array (3, cells); Gauss-Legendre
    per cell, exact away from the cells that hold a jump or a fan edge."""
    tq, wq = np.polynomial.legendre.leggauss(nq)
    a, b = edges[:-1], edges[1:]
    x = 0.5 * (a + b)[:, None] + 0.5 * (b - a)[:, None] * tq[None, :]
    rho, u, p = sample(left, right, ((x - x0) / t).ravel(), g)
    cons = np.stack([rho, rho * u, p / (g - 1.0) + 0.5 * rho * u * u])
    return np.sum(0.5 * wq[None, None, :] * cons.reshape(3, *x.shape), axis=2)
