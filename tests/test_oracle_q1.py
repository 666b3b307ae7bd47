"""Pins of the oracle's Q1 element contributions (Sec. 5.3, eq. aecQ1) and
of the low-order time derivative they use (Sec. 3, eq. weak:low1 with the
Rusanov term of eq. rusdiss; periodic, so b_i = 0).  No GPU.

Independent routes: the 1D low-order derivative of linear advection in
closed form (it is the upwind difference when dt_e is the bound of eq.
40); and, with gamma = alpha = beta = 1, the whole stage against the
target scheme m_i udot_i = -int phi_i div f_h - int phi_i (udot_h^L -
udot_i^L) written with global matrices of Q1 hat functions assembled here
from their 1D integrals (not the oracle's element tables)."""
import numpy as np
import pytest

from oracle import Mesh, Oracle, Params, Problem


def _oracle(mesh, kind, u, **prm):
    params = Params(contrib="q1", **prm)
    return Oracle(Problem(mesh, kind, velocity=(1.0, -0.6, 0.3), params=params,
                          u_min=float(u.min()), u_max=float(u.max())))


def test_q1_contributions_need_p1():
    mesh = Mesh(2, 2, (4, 4), (0.0, 0.0), (1.0, 1.0))
    with pytest.raises(ValueError):
        Oracle(Problem(mesh, "advection", params=Params(contrib="q1")))


def test_low_order_derivative_is_upwind_in_1d():
    # linear advection with speed a > 0, Q1 on a periodic 1D mesh: a_i =
    # a (u_{i+1} - u_{i-1}) / 2 and, with dt_e = h / (2 a) of eq. (40), s_i
    # = a (2 u_i - u_{i-1} - u_{i+1}) / 2, so m_i udot_i^L = -a (u_i - u_{i-1})
    n = 23
    mesh = Mesh(1, 1, (n,), (0.0,), (1.0,))
    rng = np.random.default_rng(4)
    u = rng.standard_normal((1, mesh.N))
    orc = _oracle(mesh, "advection", u)
    _, taps = orc.fe_stage(u, 1e-3)
    h = 1.0 / n
    assert np.allclose(taps["dt_e"], h / 2.0, rtol=1e-14)
    expect = -(u[0] - np.roll(u[0], 1)) / h
    assert np.allclose(taps["udot_lo"][0], expect, rtol=0, atol=1e-12 * np.max(np.abs(expect)))


def _hat_matrices(n, h):
    """periodic 1D Q1 (hat function) mass and convection int phi_i phi_j'"""
    M = np.zeros((n, n))
    C = np.zeros((n, n))
    for e in range(n):
        a, b = e, (e + 1) % n
        M[a, a] += h / 3
        M[b, b] += h / 3
        M[a, b] += h / 6
        M[b, a] += h / 6
        # phi_a = 1 - t, phi_b = t on [0, 1]: int phi_a phi_a' = -1/2, ...
        C[a, a] += -0.5
        C[a, b] += 0.5
        C[b, a] += -0.5
        C[b, b] += 0.5
    return M, C


@pytest.mark.parametrize("kind", ["advection", "kpp"])
def test_q1_stage_with_all_switches_on_is_the_target_scheme(kind):
    n0, n1 = 6, 5
    L0 = 1.0
    h = 1.0 / 6
    mesh = Mesh(2, 1, (n0, n1), (0.0, 0.0), (L0, n1 * h))
    rng = np.random.default_rng(7)
    u = 0.25 * np.pi + 3.0 * rng.random((1, mesh.N))
    orc = _oracle(mesh, kind, u, gamma_mode="one", alpha_mode="one", beta_mode="one")
    dt = 0.2 * h
    ufe, taps = orc.fe_stage(u, dt)
    Mx, Cx = _hat_matrices(n0, h)
    My, Cy = _hat_matrices(n1, h)
    M = np.kron(My, Mx)
    Dx = np.kron(My, Cx)          # int phi_i d/dx phi_j (node i0 + L0 i1)
    Dy = np.kron(Cy, Mx)
    if kind == "advection":
        fx, fy = 1.0 * u[0], -0.6 * u[0]
    else:
        fx, fy = np.sin(u[0]), np.cos(u[0])
    div = Dx @ fx + Dy @ fy       # int phi_i div f_h, f_h the nodal interpolant
    m = M.sum(axis=1)
    # the low-order derivative from per-element sums: a_i and s_i of weak:low1
    conn = mesh.connectivity()
    dte = taps["dt_e"]
    lo = np.zeros(mesh.N)
    for e in range(conn.shape[0]):
        nodes = conn[e]
        ue = u[0, nodes].mean()
        # int_K div f_h = h (mean of f_x over the +x facet - over the -x
        # facet) + h (same along y); local corners ordered x fastest
        fxe, fye = fx[nodes], fy[nodes]
        fdiv = h * ((fxe[1] + fxe[3]) - (fxe[0] + fxe[2])) / 2 + h * ((fye[2] + fye[3]) - (fye[0] + fye[1])) / 2
        mie = h * h / 4
        for i in nodes:
            lo[i] -= mie / (h * h) * fdiv + mie / dte[e] * (u[0, i] - ue)
    udotL = lo / m
    assert np.allclose(taps["udot_lo"][0], udotL, rtol=0, atol=1e-12 * np.max(np.abs(udotL)))
    target = u[0] + dt * (-div - M @ udotL + m * udotL) / m
    assert np.allclose(ufe[0], target, rtol=0, atol=1e-12 * np.max(np.abs(u)))


def test_q1_contributions_sum_to_zero_and_vanish_without_the_sensor():
    mesh = Mesh(2, 1, (7, 6), (-2.0, -2.5), (2.0, -2.5 + 6 * 4.0 / 7))
    rng = np.random.default_rng(2)
    u = np.where(rng.random((1, mesh.N)) < 0.4, 3.5 * np.pi, 0.25 * np.pi)
    orc = _oracle(mesh, "kpp", u, w_lin=0.2)
    _, taps = orc.fe_stage(u, 1e-3)
    fe = taps["fe"][0]
    assert np.max(np.abs(fe.sum(axis=-1))) <= 1e-13 * np.max(np.abs(fe))
    # the low-order derivative conserves: sum_i m_i udot_i^L = 0
    m = orc.mult * mesh.h ** 2 / mesh.nloc
    assert abs(np.sum(m * taps["udot_lo"][0])) <= 1e-13 * np.sum(m * np.abs(taps["udot_lo"][0]))
    orc0 = _oracle(mesh, "kpp", u, w_lin=0.2, gamma_mode="zero")
    ufe0, taps0 = orc0.fe_stage(u, 1e-3)
    assert np.all(taps0["fe"] == 0.0)
    # and the stage is then the low-order scheme with f = 0 on every element
    lo = Oracle(Problem(mesh, "kpp", params=Params(w_lin=0.2, gamma_mode="zero", beta_mode="zero"),
                        u_min=float(u.min()), u_max=float(u.max())))
    ufe_lo, _ = lo.fe_stage(u, 1e-3)
    assert np.allclose(ufe0, ufe_lo, rtol=0, atol=1e-14 * np.max(np.abs(u)))
