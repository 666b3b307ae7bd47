"""Pins of the oracle's Euler wave speeds against an exact Riemann solver
written from the textbook pressure function (`exact_riemann.py`, no GPU).

The facet speed lambda_ee' of the LLF flux (eq. (18)) and the subcell speeds
lambda_0i of Lemma 1 must bound the largest wave speed of the 1D Riemann
problem from above: the invariant-domain argument of Sec. 3.3 and Appendix A
needs an upper bound.  The oracle uses the two-rarefaction estimate of the
star pressure.  These tests solve the Riemann problem exactly (ideal gas,
pressure function of the left and right waves, root by bracketing) and check
  * the bound holds on many random admissible pairs, 1 < gamma <= 5/3;
  * it is exact when both nonlinear waves are rarefactions (p* <= pL, pR),
    and when the star region is a vacuum;
  * it exceeds the cheap estimate max(|v| + c) on strong shocks, where the
    cheap estimate is not a bound;
  * the normal-direction form equals the axis form of rotated states;
  * the nodal speed |v| + c of the viscosity matches closed-form states.
"""
import math

import numpy as np

from exact_riemann import extreme_speeds as exact_riemann
from oracle import physics as phys


def _cons(rho, v, p, g):
    """Conserved 1D-normal states (rho, rho v, 0, rho E) for d = 2."""
    return np.array([rho, rho * v, 0.0, p / (g - 1.0) + 0.5 * rho * v * v])


def _random_pairs(rng, n):
    g = 1.0 + (2.0 / 3.0) * (1.0 - rng.random(n))          # (1, 5/3]
    rhoL, rhoR = 10.0 ** rng.uniform(-2, 1, n), 10.0 ** rng.uniform(-2, 1, n)
    pL, pR = 10.0 ** rng.uniform(-3, 2, n), 10.0 ** rng.uniform(-3, 2, n)
    vL, vR = rng.uniform(-5, 5, n), rng.uniform(-5, 5, n)
    return g, rhoL, vL, pL, rhoR, vR, pR


def _oracle_speed(g, rhoL, vL, pL, rhoR, vR, pR):
    F = phys.Euler(2, g)
    uL = _cons(rhoL, vL, pL, g)[:, None]
    uR = _cons(rhoR, vR, pR, g)[:, None]
    return float(F.riemann_speed(uL, uR, 0)[0])


def test_speed_bounds_the_exact_riemann_solution():
    rng = np.random.default_rng(11)
    n = 10000
    g, rhoL, vL, pL, rhoR, vR, pR = _random_pairs(rng, n)
    kinds = dict(rr=0, shock=0, vacuum=0)
    for i in range(n):
        ps, sL, sR = exact_riemann(rhoL[i], vL[i], pL[i], rhoR[i], vR[i], pR[i], g[i])
        exact = max(-sL, sR, 0.0)
        got = _oracle_speed(g[i], rhoL[i], vL[i], pL[i], rhoR[i], vR[i], pR[i])
        scale = max(abs(vL[i]), abs(vR[i])) + math.sqrt(g[i] * pL[i] / rhoL[i]) \
            + math.sqrt(g[i] * pR[i] / rhoR[i])
        # upper bound (to rounding of the root and of the closed form)
        assert got >= exact - 1e-12 * scale, (i, got, exact)
        if ps == 0.0:
            kinds["vacuum"] += 1
            assert abs(got - exact) <= 1e-12 * scale
        elif ps <= min(pL[i], pR[i]):
            # two rarefactions: the estimate is the exact star pressure
            kinds["rr"] += 1
            assert abs(got - exact) <= 1e-11 * scale, (i, got, exact)
        else:
            kinds["shock"] += 1
    assert min(kinds.values()) >= 50, kinds


def test_speed_exceeds_sound_speed_estimate_on_strong_shocks():
    # a dense gas at high pressure expanding into a light gas at low
    # pressure: the shock runs into the light gas far faster than
    # max(|v| + c) of either state, so only a bound derived from the star
    # pressure is admissible
    g = 1.4
    rhoL, vL, pL, rhoR, vR, pR = 1000.0, 0.0, 1000.0, 1.0, 0.0, 0.01
    ps, sL, sR = exact_riemann(rhoL, vL, pL, rhoR, vR, pR, g)
    exact = max(-sL, sR)
    cheap = max(abs(vL) + math.sqrt(g * pL / rhoL), abs(vR) + math.sqrt(g * pR / rhoR))
    got = _oracle_speed(g, rhoL, vL, pL, rhoR, vR, pR)
    assert pR < ps < pL and exact == sR and exact > 2.5 * cheap
    assert got >= exact * (1 - 1e-14)
    # a symmetric collision: two shocks, moving apart with -sL = sR
    ps, sL, sR = exact_riemann(1.0, 2.0, 1.0, 1.0, -2.0, 1.0, g)
    assert ps > 1.0 and abs(sL + sR) <= 1e-12 * sR
    assert _oracle_speed(g, 1.0, 2.0, 1.0, 1.0, -2.0, 1.0) >= sR * (1 - 1e-14)


def test_speed_of_a_single_rarefaction_is_the_head_speed():
    # Sod-type data: p* lies between pR and pL; the left wave is a
    # rarefaction whose head moves with vL - cL
    g = 1.4
    ps, sL, sR = exact_riemann(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, g)
    assert 0.1 < ps < 1.0
    assert abs(sL - (0.0 - math.sqrt(1.4))) <= 1e-15
    got = _oracle_speed(g, 1.0, 0.0, 1.0, 0.125, 0.0, 0.1)
    assert got >= max(-sL, sR)


def test_normal_speed_is_the_axis_speed_of_rotated_states():
    rng = np.random.default_rng(5)
    F = phys.Euler(2, 1.4)
    for _ in range(200):
        rho = 10.0 ** rng.uniform(-1, 1, 2)
        v = rng.uniform(-2, 2, (2, 2))
        p = 10.0 ** rng.uniform(-2, 1, 2)
        th = rng.uniform(0, 2 * math.pi)
        n = np.array([math.cos(th), math.sin(th)])
        R = np.array([[n[0], n[1]], [-n[1], n[0]]])      # R n = e_0
        u = [np.array([rho[s], *(rho[s] * v[s]), p[s] / 0.4 + 0.5 * rho[s] * v[s] @ v[s]])
             for s in range(2)]
        ur = [np.array([rho[s], *(rho[s] * (R @ v[s])), u[s][3]]) for s in range(2)]
        a = float(F.riemann_speed_n(u[0][:, None], u[1][:, None], n)[0])
        b = float(F.riemann_speed(ur[0][:, None], ur[1][:, None], 0)[0])
        assert abs(a - b) <= 1e-13 * max(1.0, b)
        # the y-axis form is the normal form with n = e_1
        c = float(F.riemann_speed(u[0][:, None], u[1][:, None], 1)[0])
        d = float(F.riemann_speed_n(u[0][:, None], u[1][:, None], np.array([0.0, 1.0]))[0])
        assert abs(c - d) <= 1e-14 * max(1.0, c)


def test_node_speed_closed_form():
    # |v| + sqrt(gamma p / rho): rho = 4, v = (3, 4) (|v| = 5), p = 10 / 1.4
    F = phys.Euler(2, 1.4)
    rho, vx, vy, p = 4.0, 3.0, 4.0, 10.0 / 1.4
    u = np.array([rho, rho * vx, rho * vy, p / 0.4 + 0.5 * rho * 25.0])[:, None]
    assert abs(float(F.node_speed(u)[0]) - (5.0 + math.sqrt(2.5))) <= 1e-14
    assert abs(float(F.pressure(u)[0]) - p) <= 1e-14 * p
    # 3D: v = (1, 2, 2) (|v| = 3), c = 2
    F3 = phys.Euler(3, 5.0 / 3.0)
    rho, p = 1.5, 2.4                       # gamma p / rho = 4 / 1.5 * 1.5
    v = np.array([1.0, 2.0, 2.0])
    u3 = np.array([rho, *(rho * v), p / (2.0 / 3.0) + 0.5 * rho * 9.0])[:, None]
    c = math.sqrt((5.0 / 3.0) * p / rho)
    assert abs(float(F3.node_speed(u3)[0]) - (3.0 + c)) <= 1e-14 * (3.0 + c)
