"""Pins of the oracle's stage operator: closed forms, theorems and
invariants of [KHV §3, §4] (no GPU)."""
import numpy as np
import pytest

from oracle import Mesh, Oracle, Params, Problem
from paper_2509_04673_amd import workloads as W


def _lumped(orc):
    mesh = orc.mesh
    return orc.assemble(np.broadcast_to(mesh.h ** mesh.d * orc.el.lump,
                                        (1, mesh.E, mesh.nloc)).copy())[0]


def _scalar(d, p, n, kind="advection", seed=0, **prm):
    lo, hi = (0.0,) * d, (1.0,) * d
    mesh = Mesh(d, p, n, lo, hi)
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 2.0, size=(1, mesh.N))
    prob = Problem(mesh, kind, velocity=(1.0, 0.5, -0.25), params=Params(**prm),
                   u_min=float(u.min()), u_max=float(u.max()))
    return Oracle(prob), u


def _euler(d, p, n, seed=0, **prm):
    mesh = Mesh(d, p, n, (0.0,) * d, (1.0,) * d)
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.2, 2.0, mesh.N)
    vel = [rng.uniform(-1, 1, mesh.N) for _ in range(d)]
    pr = rng.uniform(0.1, 2.0, mesh.N)
    u = np.stack([rho] + [rho * v for v in vel]
                 + [pr / 0.4 + 0.5 * rho * sum(v * v for v in vel)])
    return Oracle(Problem(mesh, "euler", params=Params(**prm))), u


def test_dt_e_closed_forms():
    # P-9: dt_e = |K| / sum |S| lambda = h/2 (1D advection, |v| = 1) and
    # h/4 (2D KPP, lambda = 1)
    orc, u = _scalar(1, 2, (8,))
    _, taps = orc.fe_stage(u, 1e-4)
    assert np.allclose(taps["dt_e"], orc.mesh.h / 2, rtol=1e-15)
    mesh = Mesh(2, 2, (4, 4), (-2.0, -2.5), (2.0, 1.5))
    orc = Oracle(Problem(mesh, "kpp", u_min=0.0, u_max=12.0))
    u = np.random.default_rng(0).uniform(0.5, 11.0, (1, mesh.N))
    _, taps = orc.fe_stage(u, 1e-4)
    assert np.allclose(taps["dt_e"], mesh.h / 4, rtol=1e-15)


def test_low_order_p1_step_closed_form():
    # P-7: P1, v = 1, gamma = alpha = beta = 0, dt_e = h/2:
    # u_i^FE = (1 - 2nu) u_i + nu/4 (u_{i-2} + 3u_{i-1} + 3u_i + u_{i+1})
    orc, u = _scalar(1, 1, (16,), gamma_mode="zero", alpha_mode="zero", beta_mode="zero")
    nu = 0.3
    dt = nu * orc.mesh.h
    ufe, _ = orc.fe_stage(u, dt)
    v = u[0]
    ref = (1 - 2 * nu) * v + nu / 4 * (np.roll(v, 2) + 3 * np.roll(v, 1) + 3 * v + np.roll(v, -1))
    assert np.allclose(ufe[0], ref, atol=1e-14)


def test_high_order_bar_state_1d_p1():
    # P-8: with alpha = 1 the P1 intermediate average is the bar state (24):
    # ubar_ij = (u_i + u_j)/2 - dt_e/h (f(u_j) - f(u_i))
    orc, u = _scalar(1, 1, (16,), alpha_mode="one")
    _, taps = orc.fe_stage(u, 1e-3)
    v = u[0]
    ref = 0.5 * (v + np.roll(v, -1)) - taps["dt_e"] / orc.mesh.h * (np.roll(v, -1) - v)
    assert np.allclose(taps["ubar"][0], ref, atol=1e-14)


@pytest.mark.parametrize("d,p", [(1, 2), (2, 2), (2, 3), (3, 2)])
def test_zero_sum_of_element_contributions(d, p):
    # P-4: sum_i f_i^e = 0 [KHV eq. (47)]
    orc, u = _scalar(d, p, (4,) * d)
    _, taps = orc.fe_stage(u, 1e-4)
    scale = np.abs(taps["fe"]).max()
    assert np.abs(taps["fe"].sum(axis=-1)).max() < 1e-13 * scale


def test_zero_sum_euler():
    orc, u = _euler(2, 2, (4, 4))
    _, taps = orc.fe_stage(u, 1e-5)
    assert np.abs(taps["fe"].sum(axis=-1)).max() < 1e-13 * np.abs(taps["fe"]).max()


@pytest.mark.parametrize("kind,d,p", [("advection", 1, 2), ("advection", 2, 3),
                                      ("kpp", 2, 2), ("euler", 2, 2), ("euler", 3, 2)])
def test_equivalence_theorem(kind, d, p):
    # P-6: alpha = beta = 1 recovers the target CG-WENO scheme (10):
    # u^FE = u + dt M_C^{-1} r, whatever admissible dt_e
    if kind == "euler":
        orc, u = _euler(d, p, (4,) * d, alpha_mode="one", beta_mode="one")
    else:
        orc, u = _scalar(d, p, (4,) * d, kind=kind, alpha_mode="one", beta_mode="one")
    dt = 0.5 * orc.max_dt(u)
    ufe, taps = orc.fe_stage(u, dt)
    ref = u + dt * taps["udot"]
    assert np.abs(ufe - ref).max() < 1e-13 * np.abs(u).max()


def test_linear_flux_A_equals_G():
    # P-17: linear flux -> int grad phi_i . f(u_h) = int grad phi_i . f_h
    orc, u = _scalar(2, 3, (3, 3))
    _, taps = orc.fe_stage(u, 1e-4)
    assert np.allclose(taps["A"], taps["fgrad_h"], atol=1e-13)


def test_advection_of_c1_spline_is_exact():
    # a periodic C^1 quadratic spline: g_h = grad u_h, s_h = 0 for gamma = 1,
    # so udot is the L2 projection of -v u_h' which lies in V_h
    n = 8
    mesh = Mesh(1, 2, (n,), (0.0,), (1.0,))
    s = np.random.default_rng(2).standard_normal(n)
    u = np.zeros(mesh.N)
    for e in range(n):
        u[2 * e] = 0.5 * (s[e - 1] + s[e])
        u[2 * e + 1] = s[e]
    orc = Oracle(Problem(mesh, "advection", velocity=(1.0,), params=Params(gamma_mode="one"),
                         u_min=-10, u_max=10))
    _, taps = orc.fe_stage(u[None], 1e-4)
    h = mesh.h
    dv = np.array([(s[e] - s[e - 1]) / h for e in range(n)])
    exact = np.zeros(mesh.N)
    for e in range(n):
        exact[2 * e] = -dv[e]
        exact[2 * e + 1] = -0.5 * (dv[e] + dv[(e + 1) % n])
    assert np.allclose(taps["udot"][0], exact, atol=1e-10 * np.abs(exact).max())


def test_stabilisation_is_dissipative():
    # s_h with gamma = 0 is a Laplacian: sum_i u_i S_i = nu int |grad u_h|^2 >= 0,
    # and for linear advection sum_i u_i r_i = -sum_i u_i S_i <= 0
    orc, u = _scalar(2, 2, (5, 5), gamma_mode="zero")
    _, taps = orc.fe_stage(u, 1e-4)
    U = u[:, orc.conn]
    sS = np.sum(U * taps["S"])
    assert sS > 0
    assert np.isclose(np.sum(u * taps["r"]), -sS, rtol=1e-10)


@pytest.mark.parametrize("kind", ["advection", "kpp", "euler"])
def test_constant_state_is_preserved(kind):
    # P-3: f_i^e = 0, f^A = 0, u^FE = u for a constant state
    if kind == "euler":
        orc, _ = _euler(2, 2, (3, 3))
        u = np.tile(np.array([[1.3], [0.2], [-0.4], [2.9]]), (1, orc.mesh.N))
    else:
        orc, _ = _scalar(2, 2, (3, 3), kind=kind)
        u = np.full((1, orc.mesh.N), 0.7)
        orc.prob.u_min, orc.prob.u_max = 0.0, 1.0
    ufe, taps = orc.fe_stage(u, 0.5 * orc.max_dt(u))
    assert np.allclose(ufe, u, rtol=1e-14, atol=0)
    assert np.abs(taps["fe"]).max() < 1e-14 * np.abs(u).max() * orc.mesh.h ** 2


@pytest.mark.parametrize("kind,d,p", [("advection", 1, 2), ("advection", 2, 2), ("kpp", 2, 2),
                                      ("euler", 2, 2), ("euler", 1, 3)])
def test_conservation(kind, d, p):
    # P-5: sum_i m_i u_i is conserved by the limited stage
    if kind == "euler":
        orc, u = _euler(d, p, (5,) * d)
    else:
        orc, u = _scalar(d, p, (5,) * d, kind=kind)
    mi = _lumped(orc)
    ufe, _ = orc.fe_stage(u, 0.9 * orc.max_dt(u))
    for c in range(u.shape[0]):
        assert abs(np.sum(mi * ufe[c]) - np.sum(mi * u[c])) < 1e-14 * np.sum(mi * np.abs(u[c])) * 10


def test_idp_scalar_kpp_many_steps():
    # P-13: the limited scheme keeps u in [u_min, u_max] every stage
    wl = W.kpp2d(seed=1, n=12)
    mesh = Mesh(wl.d, wl.p, wl.n, wl.lo, wl.hi)
    prob = Problem(mesh, wl.kind, params=Params(w_lin=wl.w_lin),
                   u_min=float(wl.u0.min()), u_max=float(wl.u0.max()))
    orc = Oracle(prob)
    u, st = orc.run(wl.u0.copy(), 20, dt=2e-2)
    assert st["violations"] == 0
    assert u.min() >= prob.u_min and u.max() <= prob.u_max


def test_idp_euler_blast_positivity():
    # strong pressure jump: density and pressure stay positive (Appendix A)
    mesh = Mesh(1, 2, (24,), (0.0,), (1.0,))
    x = mesh.node_coords()[:, 0]
    pr = np.where(np.abs(x - 0.5) < 0.1, 1000.0, 0.01)
    rho = np.ones_like(x)
    u = np.stack([rho, 0 * x, pr / 0.4])
    orc = Oracle(Problem(mesh, "euler"))
    u1, st = orc.run(u, 10, cfl=0.5)
    assert st["violations"] == 0
    assert u1[0].min() > 0 and orc.prob.phys.pressure(u1).min() > 0
    # the same run with the slope limiter off leaves the admissible set
    orc_ho = Oracle(Problem(mesh, "euler", params=Params(beta_mode="one")))
    bad = 0
    v = u.copy()
    for _ in range(10):
        try:
            # leaving the admissible set makes the Riemann speeds NaN (negative
            # pressure to a fractional power): expected here, so not a warning
            with np.errstate(invalid="ignore"):
                v, st = orc_ho.run(v, 1, cfl=0.5)
        except Exception:
            bad += 1
            break
        bad += st["violations"]
        if bad:
            break
    assert bad > 0


def test_mirror_symmetry():
    # P-18: Euler data mirror-symmetric about x = 0 stay mirror-symmetric
    # (density and energy even, momentum odd)
    mesh = Mesh(1, 2, (16,), (-1.0,), (1.0,))
    x = mesh.node_coords()[:, 0]
    rho = 1.0 + 0.5 * np.exp(-10 * x ** 2)
    pr = 1.0 + (np.abs(x) < 0.3)
    u = np.stack([rho, 0 * x, pr / 0.4])
    orc = Oracle(Problem(mesh, "euler"))
    u1, _ = orc.run(u, 3, cfl=0.5)
    # node x_j = -1 + 2 j / L mirrors to node (L - j) mod L
    L = mesh.N
    perm = (L - np.arange(L)) % L
    assert np.allclose(u1[0], u1[0][perm], atol=1e-12)
    assert np.allclose(u1[2], u1[2][perm], atol=1e-12)
    assert np.allclose(u1[1], -u1[1][perm], atol=1e-12)
