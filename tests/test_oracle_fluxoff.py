"""Pins of the flux-limiter-off variant (Sec. 4.3, steps 3-4 with f = f^H):
the subcell bound of Lemma 1 [KHV eq. (37)] in closed form and its IDP
property by brute force, and the time-step reduction of the Remark after
eq. (40).  CPU only."""
import numpy as np
import pytest

from oracle import Mesh, Oracle, Params, Problem


def _orc(d, p, n, kind="advection", vel=(1.0, 0.0, 0.0), mode="subcell", bounds=(-np.inf, np.inf), L=1.0):
    mesh = Mesh(d, p, n, (0.0,) * d, (L,) * d)
    return Oracle(Problem(mesh, kind, vel, params=Params(flux_mode=mode), u_min=bounds[0], u_max=bounds[1]))


@pytest.mark.parametrize("d,p,vel,expect", [
    (1, 1, (1.0,), 1 / 4),          # s = 2, u_0 = u^e, m_0 = |K|: (1/2) min(h/2, h/2)
    (1, 2, (1.0,), 1 / 6),          # m_i = h/3, |c| = 1: min(h/3, (h/3)/2)
    (1, 3, (1.0,), 1 / 4),          # m_i = h/4: min(h/4, (h/2)/2)
    (2, 1, (1.0, 0.0), 1 / 4),      # corners |c| lambda = h/2: (1/2) min(h/2, h/2)
    (2, 2, (1.0, 0.0), 1 / 18),     # centre m_0 = h^2/9 over sum |c| lambda = 2h
])
def test_subcell_bound_closed_forms(d, p, vel, expect):
    # uniform advection: lambda_0i = |v . n_i| whatever the states
    n = (6,) * d
    orc = _orc(d, p, n, vel=vel + (0.0,) * (3 - len(vel)))
    h = orc.mesh.h
    rng = np.random.default_rng(0)
    u = rng.random((1, orc.mesh.N))
    dt = orc.subcell_dt(u[:, orc.conn], orc.fe_stage(u, 0.0)[1]["ue"])
    assert np.allclose(dt, expect * h, rtol=1e-14)


def test_subcell_bound_is_below_the_macrocell_bound():
    orc = _orc(2, 2, (5, 5), kind="kpp", bounds=(0.0, 12.0), L=4.0)
    u = np.random.default_rng(1).uniform(0, 11, (1, orc.mesh.N))
    dt_sub = orc.fe_stage(u, 0.0)[1]["dt_e"]
    lim = _orc(2, 2, (5, 5), kind="kpp", mode="limit", bounds=(0.0, 12.0), L=4.0)
    dt_cell = lim.fe_stage(u, 0.0)[1]["dt_e"]
    assert np.all(dt_sub < dt_cell)


@pytest.mark.parametrize("kind,d,p", [("advection", 2, 1), ("advection", 2, 2), ("kpp", 2, 2),
                                      ("advection", 1, 3), ("advection", 3, 2)])
def test_lemma1_idp_of_the_cell_averages_scalar(kind, d, p):
    # rough admissible data in [0, 1]: every intermediate average with
    # dt_e = dt_e^max of (37) stays in the bounds (Lemma 1)
    n = (5,) * d
    vel = (1.0, -0.7, 0.4)
    orc = _orc(d, p, n, kind=kind, vel=vel, bounds=(0.0, 1.0))
    for seed in range(4):
        u = np.random.default_rng(seed).random((1, orc.mesh.N))
        ubar = orc.fe_stage(u, 0.0)[1]["ubar"]
        assert ubar.min() >= -1e-14 and ubar.max() <= 1.0 + 1e-14


@pytest.mark.parametrize("d,p", [(1, 2), (2, 1), (2, 2), (2, 3)])
def test_lemma1_idp_of_the_cell_averages_euler(d, p):
    n = (5,) * d
    orc = _orc(d, p, n, kind="euler")
    F = orc.prob.phys
    rng = np.random.default_rng(d * 10 + p)
    for _ in range(3):
        N = orc.mesh.N
        rho = 10.0 ** rng.uniform(-2, 1, N)
        vel = [rng.uniform(-3, 3, N) for _ in range(d)]
        pr = 10.0 ** rng.uniform(-3, 1, N)
        u = np.stack([rho, *[rho * v for v in vel], pr / 0.4 + 0.5 * rho * sum(v * v for v in vel)])
        ubar = orc.fe_stage(u, 0.0)[1]["ubar"]
        assert np.all(ubar[0] > 0) and np.all(F.pressure(ubar) > 0)


def test_remark_shrink_keeps_averages_admissible_and_maximal():
    # 0/1 data: a P2 element holding (0, 0, 1) has u^e = 1/3 and, with the
    # macro-cell step h/2 and f^H = the outflow node's flux, 1/3 - 1/2 < 0
    vel = (1.0, 0.0, 0.0)
    orc = _orc(1, 2, (40,), vel=vel, mode="shrink", bounds=(0.0, 1.0))
    lim = _orc(1, 2, (40,), vel=vel, mode="limit", bounds=(0.0, 1.0))
    rng = np.random.default_rng(3)
    u = (rng.random((1, orc.mesh.N)) < 0.5).astype(float)
    taps = orc.fe_stage(u, 0.0)[1]
    dt_cell = lim.fe_stage(u, 0.0)[1]["dt_e"]
    ubar, dt = taps["ubar"][0], taps["dt_e"]
    assert ubar.min() >= -1e-14 and ubar.max() <= 1.0 + 1e-14
    assert np.all(dt <= dt_cell)
    # where the macro-cell step already gives an admissible average it is kept
    ue = taps["ue"][0]
    D = (ue - ubar) / np.where(dt > 0, dt, 1.0)
    ok = (ue - dt_cell * D >= 0.0) & (ue - dt_cell * D <= 1.0)
    assert np.all(dt[ok] == dt_cell[ok])
    assert np.any(~ok)          # the data do make some averages shrink


def test_flux_off_stage_conserves_and_keeps_constants():
    for mode in ("subcell", "shrink"):
        orc = _orc(2, 2, (5, 5), kind="kpp", mode=mode, bounds=(0.0, 12.0), L=4.0)
        u = np.full((1, orc.mesh.N), 2.5)
        dt = 0.5 * orc.max_dt(u)
        ufe, _ = orc.fe_stage(u, dt)
        assert np.max(np.abs(ufe - 2.5)) < 1e-14
        u = np.random.default_rng(5).uniform(1, 11, (1, orc.mesh.N))
        dt = 0.5 * orc.max_dt(u)
        ufe, _ = orc.fe_stage(u, dt)
        m = orc.mesh.multiplicity()
        assert abs(np.sum(m * ufe) - np.sum(m * u)) < 1e-10 * np.sum(m * u)
        assert ufe.min() >= 0.0 - 1e-12 and ufe.max() <= 12.0 + 1e-12
