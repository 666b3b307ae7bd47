"""Brute-force pins of the oracle's limiters: the flux limiter (53), the
slope limiter (54)-(55) and the Appendix A Euler limiter (no GPU)."""
import numpy as np

from oracle import Mesh, Oracle, Params, Problem


def _kpp_case(seed=0, n=6):
    mesh = Mesh(2, 2, (n, n), (-2.0, -2.5), (2.0, 1.5))
    rng = np.random.default_rng(seed)
    u = np.where(rng.random((1, mesh.N)) < 0.3, 3.5 * np.pi, 0.25 * np.pi)
    u = u + 0.3 * rng.random((1, mesh.N))
    prob = Problem(mesh, "kpp", params=Params(w_lin=0.2),
                   u_min=float(u.min()), u_max=float(u.max()))
    return Oracle(prob), u


def test_flux_limiter_is_admissible_and_maximal():
    # P-10: the clipped flux is the largest |fbar| <= |f^A| of the same sign
    # that keeps u_ee' and u_e'e in [u_min, u_max] ([KHV §4.1])
    orc, u = _kpp_case()
    prob = orc.prob
    _, taps = orc.fe_stage(u, 1e-3)
    h, d = orc.mesh.h, orc.mesh.d
    phi = h / (2 * d)
    tol = 1e-12 * max(abs(prob.u_min), abs(prob.u_max))
    limited = 0
    for k in range(d):
        hi = orc.nbr[(k, 1)]
        fA, fb = taps["fA"][k, 0], taps["fAbar"][k, 0]
        ule, ulh = taps["ubarL"][0], taps["ubarL"][0][hi]
        dte, dth = taps["dt_e"], taps["dt_e"][hi]
        assert np.all(np.abs(fb) <= np.abs(fA) + 1e-300)
        assert np.all(fb * fA >= 0)
        s1 = ule + dte * fb / phi
        s2 = ulh - dth * fb / phi
        for s in (s1, s2):
            assert np.all(s <= prob.u_max + tol) and np.all(s >= prob.u_min - tol)
        # brute force: scan f in [0, f^A] for the largest admissible value
        for i in range(fA.size):
            if fb[i] == fA[i]:
                continue
            limited += 1
            grid = np.linspace(0.0, fA[i], 20001)
            a1 = ule[i] + dte[i] * grid / phi
            a2 = ulh[i] - dth[i] * grid / phi
            ok = ((a1 <= prob.u_max + tol) & (a1 >= prob.u_min - tol)
                  & (a2 <= prob.u_max + tol) & (a2 >= prob.u_min - tol))
            best = grid[np.nonzero(ok)[0].max()]
            assert abs(best - fb[i]) <= abs(fA[i]) / 20000 * 1.01
    assert limited > 0


def test_slope_limiter_is_admissible_and_maximal():
    # P-11: beta_e is the largest value keeping every ubar + beta f_i/m_i in
    # the global bounds ([KHV eqs. (54), (55)])
    orc, u = _kpp_case(seed=3)
    prob = orc.prob
    _, taps = orc.fe_stage(u, 1e-3)
    mloc = orc.mesh.h ** 2 / orc.mesh.nloc
    fe, beta, ub = taps["fe"][0], taps["beta"], taps["ubar"][0]
    tol = 1e-12 * max(abs(prob.u_min), abs(prob.u_max))
    states = ub[:, None] + beta[:, None] * fe / mloc
    assert np.all(states <= prob.u_max + tol) and np.all(states >= prob.u_min - tol)
    assert np.all((beta >= 0) & (beta <= 1))
    lim = beta < 1
    assert lim.sum() > 0
    for e in np.nonzero(lim)[0]:
        bigger = ub[e] + min(1.0, beta[e] * (1 + 1e-9) + 1e-12) * fe[e] / mloc
        assert np.any(bigger > prob.u_max + tol * 0.5) or np.any(bigger < prob.u_min - tol * 0.5) \
            or np.any(np.isclose(states[e], prob.u_max, rtol=0, atol=tol)) \
            or np.any(np.isclose(states[e], prob.u_min, rtol=0, atol=tol))


def test_euler_appendix_a_alpha_is_admissible():
    # P-12: for alpha <= alpha_i the state ubar + alpha f/m has rho > 0 and
    # p > 0; for increments that keep the state admissible alpha_i = 1
    mesh = Mesh(2, 2, (2, 2), (0.0, 0.0), (1.0, 1.0))
    orc = Oracle(Problem(mesh, "euler"))
    F = orc.prob.phys
    rng = np.random.default_rng(11)
    n = 4000
    rho = rng.uniform(0.01, 3.0, n)
    vel = rng.uniform(-3, 3, (2, n))
    pr = rng.uniform(1e-3, 5.0, n)
    ubar = np.stack([rho, rho * vel[0], rho * vel[1], pr / 0.4 + 0.5 * rho * (vel ** 2).sum(0)])
    f = rng.standard_normal((4, n)) * rng.uniform(0.01, 20.0, n)
    m = rng.uniform(0.1, 2.0, n)
    alpha = orc._euler_alpha(ubar, f, m)
    assert np.all((alpha >= 0) & (alpha <= 1))
    for a in np.linspace(0.0, 1.0, 41):
        aa = a * alpha
        st = ubar + aa * f / m
        assert np.all(st[0] > 0)
        assert np.all(F.pressure(st) > 0)
    # some increments must actually be limited, small ones must not be
    assert np.mean(alpha < 1) > 0.1
    small = orc._euler_alpha(ubar, 1e-9 * f, m)
    assert np.all(small == 1.0)


# ---- local bounds (Sec. 4.1, 4.2: "local or global bounds") ---------------
def _kpp_local(seed=0, n=6):
    orc, u = _kpp_case(seed, n)
    orc.prob.params.bounds = "local"
    return orc, u


def test_local_bounds_contain_the_low_order_average():
    # the range of the old cell averages of K_e and its facet neighbours
    # holds the low-order average of eq. (51) (a convex combination of u^e
    # and the bar states of its facets), so the flux limiter's bounds are
    # consistent (f^max >= 0 >= f^min)
    orc, u = _kpp_local(seed=1)
    _, taps = orc.fe_stage(u, 1e-3)
    lo, hi, ubL = taps["b_lo"], taps["b_hi"], taps["ubarL"][0]
    tol = 1e-13 * np.max(np.abs(u))
    assert np.all(ubL >= lo - tol) and np.all(ubL <= hi + tol)
    # and they are the neighbourhood ranges, inside the global bounds
    ue = taps["ue"][0]
    assert np.all(lo <= ue) and np.all(hi >= ue)
    assert np.all(lo >= orc.prob.u_min) and np.all(hi <= orc.prob.u_max)
    assert np.any(hi < orc.prob.u_max) and np.any(lo > orc.prob.u_min)


def test_local_flux_limiter_is_admissible_and_maximal():
    # ubar^e of eq. (44) stays in [lo_e, hi_e]; each limited facet flux is
    # the largest |fbar| <= |f^A| keeping both sides in their own bounds
    orc, u = _kpp_local(seed=2)
    _, taps = orc.fe_stage(u, 1e-3)
    h, d = orc.mesh.h, orc.mesh.d
    phi = h / (2 * d)
    lo, hi = taps["b_lo"], taps["b_hi"]
    tol = 1e-12 * np.max(np.abs(u))
    ub = taps["ubar"][0]
    assert np.all(ub >= lo - tol) and np.all(ub <= hi + tol)
    limited = 0
    for k in range(d):
        nb = orc.nbr[(k, 1)]
        fA, fb = taps["fA"][k, 0], taps["fAbar"][k, 0]
        ule, ulh = taps["ubarL"][0], taps["ubarL"][0][nb]
        dte, dth = taps["dt_e"], taps["dt_e"][nb]
        assert np.all(np.abs(fb) <= np.abs(fA) + 1e-300) and np.all(fb * fA >= 0)
        for i in range(fA.size):
            if fb[i] == fA[i]:
                continue
            limited += 1
            grid = np.linspace(0.0, fA[i], 20001)
            a1 = ule[i] + dte[i] * grid / phi
            a2 = ulh[i] - dth[i] * grid / phi
            ok = ((a1 <= hi[i] + tol) & (a1 >= lo[i] - tol) & (a2 <= hi[nb[i]] + tol) & (a2 >= lo[nb[i]] - tol))
            best = grid[np.nonzero(ok)[0].max()]
            assert abs(best - fb[i]) <= abs(fA[i]) / 20000 * 1.01
    assert limited > 0


def test_local_slope_limiter_is_admissible_and_maximal():
    orc, u = _kpp_local(seed=3)
    _, taps = orc.fe_stage(u, 1e-3)
    mloc = orc.mesh.h ** 2 / orc.mesh.nloc
    lo, hi = taps["b_lo"], taps["b_hi"]
    ub, fe, beta = taps["ubar"][0], taps["fe"][0], taps["beta"]
    tol = 1e-12 * np.max(np.abs(u))
    states = ub[:, None] + beta[:, None] * fe / mloc
    assert np.all(states >= lo[:, None] - tol) and np.all(states <= hi[:, None] + tol)
    grid = np.linspace(0.0, 1.0, 4001)
    for e in np.nonzero(beta < 1.0)[0][:40]:
        s = ub[e] + grid[:, None] * fe[e][None, :] / mloc
        ok = np.all((s >= lo[e] - tol) & (s <= hi[e] + tol), axis=1)
        assert abs(grid[np.nonzero(ok)[0].max()] - beta[e]) <= 1.0 / 4000 * 1.01


def test_local_bounds_give_a_local_maximum_principle():
    # u_i^FE is a convex combination of u_i and the limited states of the
    # elements around node i, each in its element's bounds: per stage, the
    # new value lies in [min(u_i, min lo_e), max(u_i, max hi_e)] over e in E_i
    orc, u = _kpp_local(seed=4, n=8)
    dt = 0.5 * orc.max_dt(u)
    ufe, taps = orc.fe_stage(u, dt)
    lo_n = np.minimum(u[0], np.full(orc.mesh.N, np.inf))
    hi_n = np.maximum(u[0], np.full(orc.mesh.N, -np.inf))
    np.minimum.at(lo_n, orc.conn, np.broadcast_to(taps["b_lo"][:, None], orc.conn.shape))
    np.maximum.at(hi_n, orc.conn, np.broadcast_to(taps["b_hi"][:, None], orc.conn.shape))
    tol = 1e-12 * np.max(np.abs(u))
    assert np.all(ufe[0] >= lo_n - tol) and np.all(ufe[0] <= hi_n + tol)
    # and several stages keep the global bounds (the local ones lie inside)
    v, st = orc.run(u.copy(), 5, dt=dt)
    assert st["violations"] == 0
    assert v.min() >= orc.prob.u_min and v.max() <= orc.prob.u_max
