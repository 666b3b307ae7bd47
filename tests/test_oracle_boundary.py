"""Pins of the oracle on a non-periodic 1D line: the boundary term b_i of
eq. (bidef), the boundary facet fluxes f^partial and f^L of Sec. 4 and g_i^e
of eq. (aecb).  No GPU.

Independent routes: Galerkin exactness on global polynomials (the expected
values are Bernstein coefficients from the monomial-to-Bernstein formula,
written here), the weak form with the test function 1 (sum_i phi_i = 1:
sum_i m_i udot_i = minus the outward boundary fluxes), the low-order P1
step in closed form (first-order upwind with the inflow state), the
equivalence theorem of Sec. 4 with the boundary terms, and wall conditions
that carry no mass or energy across the ends."""
from math import comb

import numpy as np
import pytest

from oracle import Mesh, Oracle, Params, Problem


def _line(p, n, lo=0.0, hi=1.0):
    return Mesh(1, p, (n,), (lo,), (hi,), periodic=False)


def _bernstein_of_poly(mesh, coef):
    """Nodal Bernstein coefficients of the global polynomial sum_k coef[k]
    x^k on the line: per element, the Taylor coefficients c_k in t of
    u(x_e + h t), then b_a = sum_{k <= a} C(a, k) / C(p, k) c_k."""
    P = np.polynomial.Polynomial
    p, h = mesh.p, mesh.h
    out = np.zeros(mesh.N)
    for e in range(mesh.n[0]):
        c = (P(coef)(P([mesh.lo[0] + e * h, h]))).coef
        c = np.concatenate([c, np.zeros(p + 1 - len(c))])
        for a in range(p + 1):
            out[p * e + a] = sum(comb(a, k) / comb(p, k) * c[k] for k in range(a + 1))
    return out


def test_line_mesh_index_sets():
    mesh = _line(3, 5)
    assert mesh.N == 16 and mesh.E == 5
    conn = mesh.connectivity()
    assert np.array_equal(conn[0], [0, 1, 2, 3]) and np.array_equal(conn[4], [12, 13, 14, 15])
    assert np.array_equal(mesh.neighbour(0, -1), [-1, 0, 1, 2, 3])
    assert np.array_equal(mesh.neighbour(0, 1), [1, 2, 3, 4, -1])
    mult = mesh.multiplicity()
    assert mult[0] == 1 and mult[-1] == 1 and mult[3] == 2 and mult[4] == 1
    assert np.allclose(mesh.node_coords()[:, 0], np.arange(16) / 15.0)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_projected_gradient_exact_on_polynomials(p):
    # g_h = grad u_h when u_h is a global polynomial of degree <= p: no
    # periodicity is needed on the line, so any polynomial will do
    mesh = _line(p, 7, -0.5, 1.25)
    coef = np.random.default_rng(p).standard_normal(p + 1)
    u = _bernstein_of_poly(mesh, coef)[None]
    orc = Oracle(Problem(mesh, "advection", velocity=(1.0,), bc=(("state", [0.0]), ("outflow", None))))
    g = orc.projected_gradient(u)[0, 0]
    ref = _bernstein_of_poly(mesh, np.polynomial.Polynomial(coef).deriv().coef)
    assert np.allclose(g, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("p,a", [(1, 1.0), (2, 0.7), (3, -1.3)])
def test_galerkin_advection_of_polynomials_with_consistent_data(p, a):
    # u_h a global polynomial, inflow data u_hat = u_h at the inflow end,
    # gamma = 1 (so g_h = u_h' and s_h = 0): the upwind LLF flux makes b = 0
    # at both ends and udot_h is the L2 projection of -a u_h', which lies in
    # V_h, so udot is exact
    mesh = _line(p, 6)
    coef = np.random.default_rng(10 + p).standard_normal(p + 1)
    u = _bernstein_of_poly(mesh, coef)[None]
    x_in = 0 if a > 0 else -1
    bc = [("outflow", None), ("outflow", None)]
    bc[0 if a > 0 else 1] = ("state", [float(u[0, x_in])])
    orc = Oracle(Problem(mesh, "advection", velocity=(a,), bc=tuple(bc),
                         params=Params(gamma_mode="one")))
    _, taps = orc.fe_stage(u, 0.0)
    ref = -a * _bernstein_of_poly(mesh, np.polynomial.Polynomial(coef).deriv().coef)
    assert np.allclose(taps["udot"][0], ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def _lumped(orc):
    return orc.assemble(np.broadcast_to(orc.mesh.h * orc.el.lump, (1, orc.mesh.E, orc.mesh.nloc)).copy())[0]


def _euler_state(mesh, rng, g=1.4):
    rho = rng.uniform(0.3, 2.0, mesh.N)
    v = rng.uniform(-1.0, 1.0, mesh.N)
    pr = rng.uniform(0.2, 2.0, mesh.N)
    return np.stack([rho, rho * v, pr / (g - 1) + 0.5 * rho * v * v])


@pytest.mark.parametrize("kind,p", [("advection", 1), ("advection", 3), ("euler", 2)])
def test_weak_form_with_test_function_one(kind, p):
    # sum_i phi_i = 1 in eq. (weak:stab2): a(1, u_h) + b(1, u_h, u_hat) is
    # the outward boundary flux sum F(u_end, u_hat; n) and s_h(1, .) = 0, so
    # sum_i m_i udot_i = -(F_lo + F_hi) with the LLF fluxes written here
    mesh = _line(p, 9)
    rng = np.random.default_rng(3)
    if kind == "advection":
        a = 0.8
        u = rng.uniform(-1.0, 2.0, (1, mesh.N))
        st_lo, st_hi = [1.7], [-0.4]
        orc = Oracle(Problem(mesh, kind, velocity=(a,), bc=(("state", st_lo), ("state", st_hi))))

        def llf(ui, uo, n):
            return 0.5 * n * a * (ui + uo) - 0.5 * abs(a) * (uo - ui)
        F_lo = llf(u[:, 0], np.array(st_lo), -1.0)
        F_hi = llf(u[:, -1], np.array(st_hi), 1.0)
    else:
        u = _euler_state(mesh, rng)
        st_lo = [1.2, 0.3, 2.9]
        orc = Oracle(Problem(mesh, kind, bc=(("state", st_lo), ("wall", None))))
        F = orc.prob.phys

        def llf(ui, uo, n):
            lam = F.riemann_speed_n(ui, uo, np.array([n]))
            return 0.5 * n * (F.flux(ui)[0] + F.flux(uo)[0]) - 0.5 * lam * (uo - ui)
        F_lo = llf(u[:, 0], np.array(st_lo), -1.0)
        wall = u[:, -1].copy()
        wall[1] = -wall[1]
        F_hi = llf(u[:, -1], wall, 1.0)
    _, taps = orc.fe_stage(u, 0.0)
    m = _lumped(orc)
    tot = np.einsum("i,ci->c", m, taps["udot"])
    assert np.allclose(tot, -(F_lo + F_hi), rtol=1e-12, atol=1e-12 * np.abs(F_lo).max())


def test_low_order_p1_step_with_inflow_closed_form():
    # P1, a = 1 > 0, gamma = alpha = beta = 0: dt_e = h / 2 for every
    # element (the boundary facets' speeds are |a| too), the intermediate
    # averages are upwind bar states (u^{e-1} + u^e) / 2, with u^{-1} = u_hat
    # at the inflow end, and the update of eq. (49) with m_i^e = h / 2 is
    # u_i + (dt / dt_e) (mean of the bar states of E_i - u_i)
    n = 12
    mesh = _line(1, n)
    rng = np.random.default_rng(5)
    u = rng.uniform(0.0, 1.0, (1, mesh.N))
    uin = 1.5
    orc = Oracle(Problem(mesh, "advection", velocity=(1.0,), bc=(("state", [uin]), ("outflow", None)),
                         params=Params(gamma_mode="zero", alpha_mode="zero", beta_mode="zero"),
                         u_min=0.0, u_max=uin))
    h = mesh.h
    dt = 0.3 * h
    ufe, taps = orc.fe_stage(u, dt)
    assert np.allclose(taps["dt_e"], h / 2, rtol=1e-15)
    v = u[0]
    ue = 0.5 * (v[:-1] + v[1:])
    ub = 0.5 * (ue + np.concatenate([[uin], ue[:-1]]))
    assert np.allclose(taps["ubar"][0], ub, atol=1e-15)
    nu = dt / (h / 2)
    ref = v.copy()
    ref[0] = v[0] + nu * (ub[0] - v[0])
    ref[-1] = v[-1] + nu * (ub[-1] - v[-1])
    ref[1:-1] = v[1:-1] + nu * (0.5 * (ub[:-1] + ub[1:]) - v[1:-1])
    assert np.allclose(ufe[0], ref, atol=1e-14)


@pytest.mark.parametrize("kind,p", [("advection", 2), ("advection", 3), ("euler", 1), ("euler", 2)])
def test_equivalence_theorem_with_boundary_terms(kind, p):
    # Sec. 4: with alpha = beta = 1 the element contributions of eq. (45)
    # with g_i^e of eq. (aecb) recover the target scheme u + dt udot
    mesh = _line(p, 8)
    rng = np.random.default_rng(11)
    prm = Params(alpha_mode="one", beta_mode="one")
    if kind == "advection":
        u = rng.uniform(-1.0, 2.0, (1, mesh.N))
        orc = Oracle(Problem(mesh, kind, velocity=(-0.9,), params=prm, bc=(("outflow", None), ("state", [0.4]))))
    else:
        u = _euler_state(mesh, rng)
        orc = Oracle(Problem(mesh, kind, params=prm, bc=(("wall", None), ("state", [0.5, -0.2, 1.7]))))
    dt = 0.5 * orc.max_dt(u)
    ufe, taps = orc.fe_stage(u, dt)
    assert np.abs(ufe - (u + dt * taps["udot"])).max() < 1e-13 * np.abs(u).max()
    # the boundary elements' contributions still sum to zero in 1D (the
    # boundary flux is a point value, exact = lumped)
    assert np.abs(taps["fe"].sum(axis=-1)).max() < 1e-13 * np.abs(taps["fe"]).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_walls_carry_no_mass_or_energy(p):
    # the wall data reverses the momentum: the LLF fluxes F(u, u_hat; n)
    # then have zero mass and energy components, in f^partial, f^L and b,
    # so the limited stage conserves mass and energy exactly
    mesh = _line(p, 10)
    u = _euler_state(mesh, np.random.default_rng(p))
    orc = Oracle(Problem(mesh, "euler", bc=(("wall", None), ("wall", None))))
    dt = 0.4 * orc.max_dt(u)
    ufe, taps = orc.fe_stage(u, dt)
    m = _lumped(orc)
    for c in (0, 2):
        assert abs(m @ ufe[c] - m @ u[c]) <= 1e-14 * (m @ np.abs(u[c]))
    assert np.all(ufe[0] > 0) and np.all(orc.prob.phys.pressure(ufe) > 0)


def test_limited_stage_is_conservative_up_to_the_boundary_fluxes():
    # sum_i m_i (u^FE_i - u_i) = -dt sum over the two boundary facets of the
    # limited outward flux f^L - fbar^A (eqs. 44, 49; the slope limiter keeps
    # the zero sum of the 1D contributions)
    mesh = _line(2, 14)
    rng = np.random.default_rng(8)
    u = np.where(rng.random((1, mesh.N)) < 0.5, 0.0, 1.0)
    orc = Oracle(Problem(mesh, "advection", velocity=(1.0,), bc=(("state", [0.6]), ("outflow", None)),
                         u_min=0.0, u_max=1.0))
    dt = 0.5 * orc.max_dt(u)
    ufe, taps = orc.fe_stage(u, dt)
    m = _lumped(orc)
    f_hi = taps["fL"][0][0, -1] - taps["fAbar"][0][0, -1]
    # the low facet's limited outward flux f^L - fbar^A, f^L = F(u^0, u_hat; -1)
    uin = 0.6
    ue0 = taps["ue"][0, 0]
    fL_lo = 0.5 * -1.0 * (ue0 + uin) - 0.5 * (uin - ue0)
    f_lo = fL_lo - taps["fAbar_low"][0]
    assert abs(m @ ufe[0] - m @ u[0] + dt * (f_hi + f_lo)) <= 1e-14 * (m @ np.abs(u[0]))
    assert np.all(ufe >= -1e-14) and np.all(ufe <= 1.0 + 1e-14)


def test_free_stream_is_preserved():
    mesh = _line(3, 7)
    st = np.array([0.9, 0.45, 2.1])
    u = np.repeat(st[:, None], mesh.N, axis=1)
    for bc in [(("state", st), ("state", st)), (("outflow", None), ("outflow", None)),
               (("state", st), ("outflow", None))]:
        orc = Oracle(Problem(mesh, "euler", bc=bc))
        dt = 0.5 * orc.max_dt(u)
        ufe, _ = orc.fe_stage(u, dt)
        assert np.abs(ufe - u).max() <= 1e-14 * np.abs(u).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_weno_sensor_is_one_on_global_polynomials(p):
    # the boundary elements have one candidate fewer; on a global polynomial
    # every present candidate is the element's own polynomial
    mesh = _line(p, 6)
    coef = np.random.default_rng(20 + p).standard_normal(p + 1)
    u = _bernstein_of_poly(mesh, coef)[None]
    orc = Oracle(Problem(mesh, "advection", velocity=(1.0,), bc=(("outflow", None), ("outflow", None))))
    gam = orc.weno_gamma(u[:, orc.conn])
    assert np.all(gam > 1.0 - 1e-6), gam


def test_local_bounds_include_the_boundary_data():
    # the inflow state lies above every cell average: the local bounds of
    # element 0 reach it, and the low-order averages lie in the bounds
    mesh = _line(2, 10)
    rng = np.random.default_rng(2)
    u = rng.uniform(0.0, 1.0, (1, mesh.N))
    orc = Oracle(Problem(mesh, "advection", velocity=(1.0,), bc=(("state", [3.0]), ("outflow", None)),
                         params=Params(bounds="local"), u_min=0.0, u_max=3.0))
    _, taps = orc.fe_stage(u, 1e-3)
    assert taps["b_hi"][0] == 3.0 and np.all(taps["b_hi"][1:] <= 1.0)
    tol = 1e-14
    assert np.all(taps["ubarL"][0] >= taps["b_lo"] - tol) and np.all(taps["ubarL"][0] <= taps["b_hi"] + tol)
    assert np.all(taps["ubar"][0] >= taps["b_lo"] - tol) and np.all(taps["ubar"][0] <= taps["b_hi"] + tol)


def test_subcell_and_q1_rejected_on_lines():
    mesh = _line(1, 4)
    for prm in (Params(flux_mode="subcell"), Params(contrib="q1")):
        with pytest.raises(ValueError):
            Oracle(Problem(mesh, "advection", velocity=(1.0,), params=prm,
                           bc=(("outflow", None), ("outflow", None))))


def _sod(p, n):
    mesh = _line(p, n)
    x = mesh.node_coords()[:, 0]
    left = x < 0.25
    rho = np.where(left, 1.0, 0.125)
    v = np.where(left, 0.75, 0.0)
    pr = np.where(left, 1.0, 0.1)
    u = np.stack([rho, rho * v, pr / 0.4 + 0.5 * rho * v * v])
    return mesh, u, u[:, 0].copy(), u[:, -1].copy()


@pytest.mark.parametrize("p", [1, 2])
def test_modified_sod_run_stays_admissible(p):
    # Sec. 5.2.1: supersonic inlet data at x = 0, the right initial state at
    # x = 1; limited run keeps rho, p > 0 and mass changes only by the
    # boundary fluxes (here: inflow at the left, none at the right)
    mesh, u, sl, sr = _sod(p, 64 // p)
    orc = Oracle(Problem(mesh, "euler", bc=(("state", sl), ("state", sr))))
    un, st = orc.run(u, 15, cfl=0.5)
    assert st["violations"] == 0
    assert np.all(un[0] > 0) and np.all(orc.prob.phys.pressure(un) > 0)
    m = _lumped(orc)
    assert m @ un[0] > m @ u[0]            # mass flows in through the inlet


@pytest.mark.parametrize("p,kind", [(2, "advection"), (3, "advection"), (2, "euler")])
def test_interior_of_the_line_is_the_periodic_scheme(p, kind):
    # data that is constant (to far below rounding) near both ends: the
    # line with matching boundary data and the periodic mesh give the same
    # run, since the boundary terms vanish and the line's mass and gradient
    # operators differ from the periodic ones only near the ends (the
    # inverse mass rows decay by ~1e-17 over 30-60 nodes: the bump stays
    # 120 nodes away from the ends)
    n = 240 // p
    line = _line(p, n)
    per = Mesh(1, p, (n,), (0.0,), (1.0,))
    def init(mesh):
        x = mesh.node_coords()[:, 0]
        bump = np.exp(-300.0 * (x - 0.5) ** 2)
        if kind == "advection":
            return bump[None]
        rho = 1.0 + 0.5 * bump
        return np.stack([rho, 0.3 * rho, 1.0 / 0.4 + 0.5 * 0.09 * rho])
    ul = init(line)
    up = init(per)
    if kind == "advection":
        kw = dict(velocity=(1.0,), u_min=0.0, u_max=1.0)
        bc = (("state", [0.0]), ("outflow", None))
    else:
        kw = {}
        bc = (("state", ul[:, 0]), ("state", ul[:, -1]))
    ol = Oracle(Problem(line, kind, bc=bc, **kw))
    op = Oracle(Problem(per, kind, **kw))
    dt = 0.4 * op.max_dt(up)
    rl, _ = ol.run(ul, 6, dt=dt)
    rp, _ = op.run(up, 6, dt=dt)
    assert np.abs(rl[:, :-1] - rp).max() <= 1e-13 * np.abs(up).max()
