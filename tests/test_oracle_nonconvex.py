"""Pins of the oracle's 1D nonconvex flux (Sec. 5.1.2, eq. 1dkpp-flux) and
of the scheme on the paper's Riemann problem with inflow (no GPU).

Independent routes: the flux's stated properties (C^1 at u = 1/2, concave
below, convex above) checked numerically; the speed bound against brute-
force sampling of |f'| between the states; and the exact entropy solution
of u_0 = chi_{x >= 1/4} with inflow u(0, t) = 0, derived here from the lower
convex envelope of f on [0, 1]: a shock from 0 to u* = sqrt(3/8), where the
chord from (0, 0) touches the convex branch (f'(u*) = f(u*) / u*), moving at
s = u* - 1/2, followed by the rarefaction u = 1/2 + (x - 1/4)/t up to
x = 1/4 + t/2."""
import numpy as np
import pytest

from oracle import Mesh, Oracle, Params, Problem
from oracle.physics import NonConvex


def test_flux_is_c1_concave_then_convex():
    F = NonConvex(1)
    f = lambda v: F.flux(np.asarray(v, dtype=float))[0]
    e = 1e-7
    assert abs(f(0.5) - 1.0 / 16.0) < 1e-15 and abs(f(0.5 + 1e-12) - 1.0 / 16.0) < 1e-12
    # one-sided difference quotients at 1/2 both vanish (f' continuous)
    assert abs((f(0.5) - f(0.5 - e)) / e) < 1e-6 and abs((f(0.5 + e) - f(0.5)) / e) < 1e-6
    u = np.linspace(-1.0, 2.0, 3001)
    d2 = f(u[2:]) - 2 * f(u[1:-1]) + f(u[:-2])
    mid = u[1:-1]
    assert np.all(d2[mid < 0.5 - 2e-3] < 0) and np.all(d2[mid > 0.5 + 2e-3] > 0)
    # f is piecewise quadratic: central differences give f' exactly away
    # from the kink
    away = np.abs(mid - 0.5) > 2e-3
    cd = (f(u[2:]) - f(u[:-2])) / (u[2] - u[0])
    assert np.allclose(F.dflux(mid)[away], cd[away], atol=1e-9)


def test_riemann_speed_bounds_f_prime_between_the_states():
    F = NonConvex(1)
    rng = np.random.default_rng(0)
    for _ in range(2000):
        a, b = rng.uniform(-1.0, 2.0, 2)
        w = np.linspace(min(a, b), max(a, b), 201)
        brute = np.max(np.abs(F.dflux(w)))
        lam = F.riemann_speed(np.array([a]), np.array([b]), 0)
        assert brute <= lam + 1e-15 and lam <= brute + 1e-15


def exact(x, t):
    us = np.sqrt(3.0 / 8.0)
    xs = 0.25 + (us - 0.5) * t
    xr = 0.25 + 0.5 * t
    return np.where(x < xs, 0.0, np.where(x < xr, 0.5 + (x - 0.25) / t, 1.0))


def _run(n, p, T=1.0):
    mesh = Mesh(1, p, (n,), (0.0,), (1.0,), periodic=False)
    x = mesh.node_coords()[:, 0]
    u = (x >= 0.25).astype(float)[None]
    orc = Oracle(Problem(mesh, "nonconvex", params=Params(), u_min=0.0, u_max=1.0,
                         bc=(("state", [0.0]), ("outflow", None))))
    dt0 = 0.5 * orc.max_dt(u)
    nsteps = int(np.ceil(T / dt0))
    un, st = orc.run(u, nsteps, dt=T / nsteps)
    # cell averages against the exact cell averages (Gauss, 8 points; the
    # exact solution is piecewise linear, the kink cells converge anyway)
    tq, wq = np.polynomial.legendre.leggauss(8)
    xl = mesh.h * np.arange(n)
    ex = np.array([np.sum(wq * exact(a + mesh.h * (tq + 1) / 2, T)) / 2 for a in xl])
    U = un[0][mesh.connectivity()]
    return mesh.h * np.sum(np.abs(U.mean(axis=1) - ex)), st, un


def test_exact_entropy_solution_sanity():
    us = np.sqrt(3.0 / 8.0)
    F = NonConvex(1)
    # the chord from (0, 0) is tangent at u*: f(u*) / u* = f'(u*)
    assert abs(F.flux(np.array(us))[0] / us - F.dflux(np.array(us))) < 1e-15
    # the solution is continuous at the rarefaction's tail (the shock's
    # right state) and head
    t = 1.0
    xs = 0.25 + (us - 0.5) * t
    assert abs(exact(np.array([xs + 1e-12]), t)[0] - us) < 1e-10
    assert abs(exact(np.array([0.75 - 1e-12]), t)[0] - 1.0) < 1e-10


@pytest.mark.parametrize("p", [1, 2])
def test_limited_scheme_converges_to_the_entropy_solution(p):
    # N_h = 129 as in the paper and twice that: the L1 error at t = 1 drops
    # with h, stays small, and the scheme keeps [0, 1]
    e1, st1, u1 = _run(128 // p, p)
    e2, st2, _ = _run(256 // p, p)
    assert e1 < 1.5e-2 and e2 < 0.75 * e1, (e1, e2)
    assert st1["violations"] == 0 and st2["violations"] == 0
    assert u1.min() >= -1e-14 and u1.max() <= 1.0 + 1e-14
