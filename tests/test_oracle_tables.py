"""Pins of the oracle's Bernstein tables, consistent-mass solve and projected
gradient against closed forms and brute force (no GPU)."""
from fractions import Fraction
from math import comb

import numpy as np
import pytest

from oracle import Mesh, Oracle, Problem
from oracle import bernstein as bz


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_partition_of_unity_and_nonnegativity(p):
    # [KHV §2.1]: nonnegative basis forming a partition of unity
    t = np.linspace(0.0, 1.0, 101)
    V = bz.basis_values(p, t)
    assert np.all(V >= -1e-15)
    assert np.allclose(V.sum(axis=1), 1.0, atol=1e-14)
    # derivatives of a partition of unity sum to zero
    assert np.allclose(bz.basis_derivs(p, t).sum(axis=1), 0.0, atol=1e-12)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_mass_closed_form_and_lumped_mass(p):
    # textbook: int B_a B_b = C(p,a) C(p,b) / ((2p+1) C(2p, a+b));
    # int B_a = 1/(p+1) so m_i^e = |K_e| / |N_e| ([KHV §3])
    ex = bz.exact_tables(p)
    for a in range(p + 1):
        assert ex["lump"][a] == Fraction(1, p + 1)
        for b in range(p + 1):
            assert ex["mass"][a][b] == Fraction(comb(p, a) * comb(p, b),
                                                (2 * p + 1) * comb(2 * p, a + b))
        assert sum(ex["mass"][a]) == Fraction(1, p + 1)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_integration_by_parts_identity(p):
    # int B_a B_b' + int B_a' B_b = [B_a B_b]_0^1 catches sign/transpose slips
    ex = bz.exact_tables(p)
    for a in range(p + 1):
        for b in range(p + 1):
            bnd = int(a == p and b == p) - int(a == 0 and b == 0)
            assert ex["cdiv"][a][b] + ex["cgrad"][a][b] == bnd
            assert ex["cgrad"][a][b] == ex["cdiv"][b][a]


@pytest.mark.parametrize("p", [1, 2, 3])
def test_tables_against_brute_force_quadrature(p):
    t, w = bz.gauss(20)
    B, D = bz.basis_values(p, t), bz.basis_derivs(p, t)
    T = bz.tables(p)
    assert np.allclose(T["mass"], B.T @ (w[:, None] * B), atol=1e-15)
    assert np.allclose(T["cdiv"], B.T @ (w[:, None] * D), atol=1e-14)
    assert np.allclose(T["stiff"], D.T @ (w[:, None] * D), atol=1e-13)
    # derivative table against a central finite difference of the values
    hh = 1e-6
    fd = (bz.basis_values(p, t + hh) - bz.basis_values(p, t - hh)) / (2 * hh)
    assert np.allclose(D, fd, atol=1e-7)


def test_bernstein_derivative_via_differences():
    # d/dt sum c_a B_a^p = p sum (c_{a+1} - c_a) B_a^{p-1}
    rng = np.random.default_rng(1)
    t = np.linspace(-1.0, 2.0, 17)
    for p in (1, 2, 3, 4):
        c = rng.standard_normal(p + 1)
        lhs = bz.basis_derivs(p, t) @ c
        rhs = bz.derivative_factor(p, 1) * (bz.basis_values(p - 1, t) @ np.diff(c))
        assert np.allclose(lhs, rhs, atol=1e-12)


def _global_basis_values(mesh, pts):
    """Brute force: value of every global basis function at points (P, d),
    built pointwise from the element that contains each point."""
    d, p, h = mesh.d, mesh.p, mesh.h
    conn = mesh.connectivity()
    P = pts.shape[0]
    V = np.zeros((P, mesh.N))
    G = [np.zeros((P, mesh.N)) for _ in range(d)]
    eidx = np.floor((pts - np.array(mesh.lo)) / h).astype(int)
    loc = (pts - np.array(mesh.lo)) / h - eidx
    eid = sum(eidx[:, k] * mesh.elem_stride[k] for k in range(d))
    aidx = mesh.local_index()
    for j in range(mesh.nloc):
        val = np.ones(P)
        ders = [np.ones(P) for _ in range(d)]
        for k in range(d):
            bv = bz.basis_values(p, loc[:, k])[:, aidx[j, k]]
            bd = bz.basis_derivs(p, loc[:, k])[:, aidx[j, k]] / h
            val = val * bv
            for kk in range(d):
                ders[kk] = ders[kk] * (bd if kk == k else bv)
        cols = conn[eid, j]
        np.add.at(V, (np.arange(P), cols), val)
        for kk in range(d):
            np.add.at(G[kk], (np.arange(P), cols), ders[kk])
    return V, G


def _fine_quadrature(mesh, nq=8):
    t, w = bz.gauss(nq)
    d, h = mesh.d, mesh.h
    pts, wts = [], []
    eidx = mesh.element_index()
    grids = np.meshgrid(*([t] * d), indexing="ij")
    wg = np.ones(())
    for _ in range(d):
        wg = np.multiply.outer(wg, w)
    loc = np.stack([g.ravel() for g in grids], axis=1)
    for e in range(mesh.E):
        pts.append(np.array(mesh.lo) + h * (eidx[e] + loc))
        wts.append(wg.ravel() * h ** d)
    return np.concatenate(pts), np.concatenate(wts)


@pytest.mark.parametrize("d,p,n", [(1, 2, (5,)), (2, 2, (3, 4)), (2, 3, (3, 3)), (3, 2, (2, 2, 3))])
def test_consistent_mass_solve_matches_dense_global_assembly(d, p, n):
    # P-2: M_C assembled by brute-force quadrature of global basis functions
    mesh = Mesh(d, p, n, (0.0,) * d, tuple(0.5 * nk for nk in n))
    orc = Oracle(Problem(mesh, "advection"))
    pts, wts = _fine_quadrature(mesh)
    V, _ = _global_basis_values(mesh, pts)
    MC = V.T @ (wts[:, None] * V)
    b = np.random.default_rng(0).standard_normal((2, mesh.N))
    x = orc.solve_consistent_mass(b)
    assert np.allclose(MC @ x.T, b.T, atol=1e-11 * np.abs(b).max())


@pytest.mark.parametrize("d,p,n", [(1, 3, (4,)), (2, 2, (3, 4))])
def test_projected_gradient_against_brute_force(d, p, n):
    # g_h = M_C^{-1} (int phi_i grad u_h) computed with dense brute force
    mesh = Mesh(d, p, n, (0.0,) * d, tuple(0.25 * nk for nk in n))
    orc = Oracle(Problem(mesh, "advection"))
    u = np.random.default_rng(3).standard_normal((1, mesh.N))
    pts, wts = _fine_quadrature(mesh)
    V, G = _global_basis_values(mesh, pts)
    MC = V.T @ (wts[:, None] * V)
    g = orc.projected_gradient(u)
    for k in range(d):
        bk = V.T @ (wts * (G[k] @ u[0]))
        assert np.allclose(g[k, 0], np.linalg.solve(MC, bk), atol=1e-10)


def test_projected_gradient_of_c1_spline_is_exact():
    # a periodic C^1 quadratic spline has grad u_h in V_h, so g_h = grad u_h
    n, p = 8, 2
    mesh = Mesh(1, p, (n,), (0.0,), (1.0,))
    rng = np.random.default_rng(5)
    s = rng.standard_normal(n)          # B-spline control points (periodic)
    # Bernstein coefficients of a uniform quadratic B-spline on each cell:
    # c0 = (s_{e-1}+s_e)/2, c1 = s_e, c2 = (s_e+s_{e+1})/2
    u = np.zeros(mesh.N)
    for e in range(n):
        u[2 * e] = 0.5 * (s[e - 1] + s[e])
        u[2 * e + 1] = s[e]
    orc = Oracle(Problem(mesh, "advection"))
    g = orc.projected_gradient(u[None])[0, 0]
    h = mesh.h
    # derivative of the spline is piecewise linear: at vertex 2e it is
    # (s_e - s_{e-1})/h; on the cell it is linear, so its degree-2 Bernstein
    # coefficients are the vertex values and their mean
    dv = np.array([(s[e] - s[e - 1]) / h for e in range(n)])
    exact = np.zeros(mesh.N)
    for e in range(n):
        exact[2 * e] = dv[e]
        exact[2 * e + 1] = 0.5 * (dv[e] + dv[(e + 1) % n])
    assert np.allclose(g, exact, atol=1e-11 * np.abs(exact).max())
