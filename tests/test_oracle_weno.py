"""Pins of the oracle's WENO sensor [KHV eqs. (7), (8)] (no GPU)."""
import numpy as np
import pytest

from oracle import Mesh, Oracle, Params, Problem
from oracle import bernstein as bz


def _interp_coeffs(p, f1d_vals_fn):
    """Bernstein coefficients of a polynomial on [0,1] by interpolation at
    p+1 equispaced points (numpy solve; independent of the oracle)."""
    t = np.linspace(0.0, 1.0, p + 1)
    V = bz.basis_values(p, t)
    return np.linalg.solve(V, f1d_vals_fn(t))


def _oracle(d, p, n, w_lin=1e-3, eps=1e-12, kind="advection"):
    mesh = Mesh(d, p, n, (0.0,) * d, tuple(float(nk) for nk in n))
    return Oracle(Problem(mesh, kind, params=Params(w_lin=w_lin, eps=eps)))


def test_seminorm_closed_forms_1d():
    # P-15: ||t||^2 = int 1 = 1 and ||t^2||^2 = int (2t)^2 + int 2^2 = 16/3 (p = 2)
    orc = _oracle(1, 2, (3,))
    for coeffs, exact in (([0.0, 0.5, 1.0], 1.0), ([0.0, 0.0, 1.0], 16.0 / 3.0)):
        U = np.tile(np.array(coeffs), (3, 1))[None]     # (m, E, nloc)
        beta = orc.weno_parts(U)["beta"][0, 0]
        assert np.allclose(beta, exact, rtol=1e-14)


def test_seminorm_closed_form_2d_xy():
    # v = x y on the reference square, p = 2: |k|=1 gives int y^2 + int x^2
    # = 2/3, |k|=2 gives int (d_xy v)^2 = 1 -> 5/3
    p = 2
    orc = _oracle(2, p, (2, 2))
    cx = _interp_coeffs(p, lambda t: t)
    C = np.outer(cx, cx)                 # [a_y, a_x]
    U = np.tile(C.ravel(), (4, 1))[None]
    beta = orc.weno_parts(U)["beta"][0, 0]
    assert np.allclose(beta, 5.0 / 3.0, rtol=1e-14)


def test_seminorm_zero_on_constants_and_scale_free():
    orc = _oracle(2, 3, (3, 3))
    U = np.full((1, 9, 16), 2.7)
    parts = orc.weno_parts(U)
    assert np.all(parts["beta"] == 0.0) and np.all(parts["dev"] == 0.0)
    assert np.all(parts["gamma"] == 1.0)
    # semi-norm (8) is h-free on cubes: same coefficients, other cell size
    rng = np.random.default_rng(0)
    V = rng.standard_normal((1, 9, 16))
    small = Oracle(Problem(Mesh(2, 3, (3, 3), (0.0, 0.0), (0.03, 0.03)), "advection"))
    assert np.allclose(orc.weno_parts(V)["beta"], small.weno_parts(V)["beta"], rtol=1e-13)


@pytest.mark.parametrize("d,p", [(1, 2), (1, 3), (2, 2), (2, 3)])
def test_gamma_is_one_on_a_global_polynomial(d, p):
    # P-14: all candidates equal the global polynomial -> deviation 0 -> gamma 1
    n = (6,) * d
    orc = _oracle(d, p, n)
    mesh = orc.mesh
    rng = np.random.default_rng(d * 10 + p)
    coef = rng.standard_normal((p + 1,) * d)          # monomial coefficients

    def poly(x):                                      # x: (P, d) physical
        out = np.zeros(x.shape[0])
        for idx in np.ndindex(*coef.shape):
            term = coef[idx] * np.ones(x.shape[0])
            for k in range(d):
                term = term * (x[:, k] / 6.0) ** idx[k]
            out += term
        return out

    # Bernstein coefficients per element by tensor interpolation (numpy solve)
    t = np.linspace(0.0, 1.0, p + 1)
    Vinv = np.linalg.inv(bz.basis_values(p, t))
    aidx = mesh.local_index()
    eidx = mesh.element_index()
    U = np.zeros((1, mesh.E, mesh.nloc))
    for e in range(mesh.E):
        pts = np.array([[eidx[e, k] + t[aidx[j, k]] for k in range(d)] for j in range(mesh.nloc)])
        vals = poly(pts).reshape((p + 1,) * d)       # C order: last axis = axis 0
        C = vals
        for k in range(d):
            C = np.moveaxis(np.tensordot(Vinv, C, axes=([1], [C.ndim - 1 - k])), 0, C.ndim - 1 - k)
        U[0, e] = C.ravel()
    gam = orc.weno_parts(U)["gamma"][0]
    # elements away from the periodic seam see the same global polynomial
    inner = np.all((eidx >= 1) & (eidx <= 4), axis=1)
    assert np.all(gam[inner] > 1.0 - 1e-9)


def test_gamma_range_and_jump_detection():
    orc = _oracle(1, 2, (32,))
    x = orc.mesh.node_coords()[:, 0] / 32.0
    u = np.where((x > 0.3) & (x < 0.6), 1.0, 0.0) + 0.1 * np.sin(2 * np.pi * x)
    gam = orc.weno_parts(u[None][:, orc.conn])["gamma"][0]
    assert np.all((gam >= 0.0) & (gam <= 1.0))
    # the elements containing the jumps are flagged, smooth ones are not
    xe = (np.arange(32) + 0.5) / 32
    jump = (np.abs(xe - 0.3) < 1.0 / 32) | (np.abs(xe - 0.6) < 1.0 / 32)
    assert gam[jump].min() < 0.5
    far = (np.abs(xe - 0.3) > 3.0 / 32) & (np.abs(xe - 0.6) > 3.0 / 32)
    assert gam[far].min() > 0.9


def test_gamma_affine_invariance():
    # with eps -> 0 the sensor only sees ratios of semi-norms
    orc = _oracle(2, 2, (5, 5), eps=1e-300)
    rng = np.random.default_rng(7)
    U = rng.standard_normal((1, 25, 9))
    g1 = orc.weno_parts(U)["gamma"]
    g2 = orc.weno_parts(3.5 * U - 2.0)["gamma"]
    assert np.allclose(g1, g2, atol=1e-12)
    assert np.all((g1 >= 0) & (g1 <= 1))


def test_constant_element_next_to_varying_neighbour():
    # regularised 0/0 reading: a constant element has zero own semi-norm and
    # the sensor ratio is taken against (||u||^2 + eps)^(1/2); it is smooth
    # (gamma ~ 1), continuous in the data, and the varying element is not
    orc = _oracle(1, 2, (4,))
    U = np.zeros((1, 4, 3))
    U[0, 1] = [0.0, 0.3, 1.0]
    gam = orc.weno_parts(U)["gamma"][0]
    assert gam[0] > 1 - 1e-6 and gam[2] > 1 - 1e-6
    assert gam[3] == 1.0        # itself and both neighbours constant
    assert gam[1] < 0.5
    # continuity: a 1-ulp perturbation of a constant element moves gamma by
    # at most |u| ulp / sqrt(eps)
    V = U.copy()
    V[0, 3] = [0.0, 2.0 ** -1074, 0.0]
    g2 = orc.weno_parts(V)["gamma"][0]
    assert np.max(np.abs(g2 - gam)) < 1e-9
