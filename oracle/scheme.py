"""One explicit SSP-RK stage of the limited CG-WENO scheme: the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Plain float64 numpy, vectorised over elements with dense element matrices
built from the exact tables of ``oracle.bernstein``; global sums use
``np.add.at`` in element order; the consistent mass matrix is inverted with a
dense LU factorisation per axis.  The stage follows the five-step algorithm
of [KHV §4.3] in the paper's order and notation on a uniform periodic box
(so the boundary terms b_i and g_i^e vanish, [KHV §3.1, §4]) or on a
non-periodic 1D line with weakly imposed boundary data (b_i of eq. bidef,
f^partial of Sec. 4, g_i^e of eq. aecb).

Readings of points the paper leaves open:
  * g_h is the consistent L2 projection of grad u_h, solved exactly.
  * lambda_e is the largest nodal speed of the element, h_e the cell edge.
  * WENO candidates: v_0 = u_h^e; one candidate per facet neighbour, the
    neighbour's polynomial extended into K_e (its cell average is
    irrelevant: the semi-norm (8) has no zero-order term); r = 2,
    eps = 1e-12; gamma_e of a system is the minimum over components;
    the ratio in (7) is 0/0 on constant elements and is regularised as
    ||u - u*||_e / (||u||_e^2 + eps)^(1/2) with the weights' epsilon.
  * The element integral of grad(phi_i) . f(u_h) uses (p+1)^d Gauss points.
  * The flux limiter is on with pseudo time steps (40); Euler facet pairs use
    Appendix A with the increments the states u_ee', u_e'e actually receive.
  * Non-periodic lines (1D): the boundary data u_hat is a prescribed state,
    the interior state itself (outflow) or, for Euler, the mirror state with
    reversed momentum (wall); u_hat^{e'} of the low-order boundary flux is
    that data for the state u^e; a WENO candidate across a boundary facet is
    absent (weight 0); the flux limiter of a boundary facet keeps only its
    element's bounds (eq. 53, e' > E_h); local bounds include u_hat^{e'}.
  * Strict positivity margin eps_pos in the Appendix A limiters; slope
    limiter ratios of (55) are clipped to [0, 1]; a scalar stage result that
    leaves [u_min, u_max] by no more than a few ulps of rounding is clamped
    back and counted, larger excursions are left and counted as violations.
"""
from dataclasses import dataclass, field
from functools import cached_property

import numpy as np
import scipy.linalg

from . import bernstein as bz
from . import physics as phys
from .mesh import Mesh, multi_indices


@dataclass
class Params:
    q: float = 1.0              # steepening exponent of (7); q = 1 [KHV §5]
    r: float = 2.0              # exponent of the WENO weights
    eps: float = 1e-12          # epsilon of the WENO weights
    w_lin: float = 1e-3         # linear weight of each neighbour candidate
    gamma_mode: str = "weno"    # "weno" | "zero" | "one"   (LO/HO switches)
    alpha_mode: str = "limit"   # "limit" | "one" | "zero"  flux limiter
    beta_mode: str = "limit"    # "limit" | "one" | "zero"  slope limiter
    eps_pos: float = 1e-10      # strict-positivity margin (Euler)
    clamp_ulps: float = 64.0    # round-off clamp width, in ulps of max|bound|
    # intermediate cell averages [KHV Sec. 4.3, step 3]: "limit" = flux
    # limiter with dt_e of eq. (40); "subcell" = no flux limiter (f = f^H)
    # with dt_e of eq. (37); "shrink" = no flux limiter, dt_e of eq. (40)
    # reduced until ubar^e is admissible (the Remark after eq. (40))
    flux_mode: str = "limit"
    # bounds of the scalar limiters [KHV Sec. 4.1, 4.2, "local or global
    # bounds"]: "global" = [u_min, u_max]; "local" = per element, the range
    # of the old cell averages of the element and its facet neighbours,
    # imposed on ubar^e (flux limiter) and on the limited states of the
    # element's nodes (slope limiter)
    bounds: str = "global"
    # antidiffusive element contributions: "aec" = [KHV eq. (45)]; "q1" =
    # the Q1 form of [KHV Sec. 5.3] (p = 1), gamma_e (m_i^e (u_i - u^e) -
    # dt_e [int (phi_i - m_i^e/|K|) div f_h + int phi_i (udot_h^L -
    # udot_i^L)]), with udot^L the time derivative of the low-order scheme
    # of [KHV Sec. 3] (eq. weak:low1 with the Rusanov term, b_i = 0)
    contrib: str = "aec"


@dataclass
class Problem:
    mesh: Mesh
    kind: str
    velocity: tuple = (1.0, 0.0, 0.0)
    gamma_gas: float = 1.4
    params: Params = field(default_factory=Params)
    u_min: float = -np.inf      # global bounds (scalar problems)
    u_max: float = np.inf
    # boundary conditions of a non-periodic line [KHV eq. (ibvp)]: one
    # (kind, state) pair per end (lo, hi); kind "state" (u_hat = the given
    # conserved state), "outflow" (u_hat = u) or "wall" (Euler: u_hat = the
    # state with reversed momentum)
    bc: tuple = None

    def __post_init__(self):
        self.phys = phys.make(self.kind, self.mesh.d, self.velocity, self.gamma_gas)
        self.m = self.phys.m
        if self.mesh.periodic:
            assert self.bc is None, "boundary conditions need a non-periodic mesh"
        else:
            assert self.bc is not None and len(self.bc) == 2
            for kind, state in self.bc:
                assert kind in ("state", "outflow", "wall"), kind
                assert kind != "wall" or self.kind == "euler", "walls are an Euler condition"
                assert kind != "state" or len(state) == self.m


# ---------------------------------------------------------------------------
# element matrices (Kronecker products of the exact 1D tables)
# ---------------------------------------------------------------------------
def _kron_axes(mats):
    """d-dim operator from per-axis 1D matrices (mats[k] acts on axis k);
    local ids have axis 0 fastest, so axis 0 is the last Kronecker factor."""
    out = np.ones((1, 1))
    for k in reversed(range(len(mats))):
        out = np.kron(out, mats[k])
    return out


class Element:
    def __init__(self, d, p):
        self.d, self.p = d, p
        t1 = bz.tables(p)
        self.t1 = t1
        nq1 = p + 1
        tq, wq = bz.gauss(nq1)
        Bq = bz.basis_values(p, tq)     # (q, a)
        Dq = bz.basis_derivs(p, tq)
        self.mass = _kron_axes([t1["mass"]] * d)
        self.cdiv, self.cgrad, self.stiff, self.dvq = [], [], [], []
        for k in range(d):
            pick = lambda A, B: [A if j == k else B for j in range(d)]
            self.cdiv.append(_kron_axes(pick(t1["cdiv"], t1["mass"])))
            self.cgrad.append(_kron_axes(pick(t1["cgrad"], t1["mass"])))
            self.stiff.append(_kron_axes(pick(t1["stiff"], t1["mass"])))
            self.dvq.append(_kron_axes(pick(Dq, Bq)))
        self.vq = _kron_axes([Bq] * d)
        self.wq = _kron_axes([wq[None, :]] * d)[0]
        # int over [0,1]^d of d/dxi_k phi_j : (B_j(1) - B_j(0)) along k
        end = np.zeros(p + 1)
        end[p], end[0] = 1.0, -1.0
        self.int_dphi = [_kron_axes([end[None, :] if j == k else t1["lump"][None, :]
                                     for j in range(d)])[0] for k in range(d)]
        self.lump = _kron_axes([t1["lump"][None, :]] * d)[0]
        self.tq, self.wq1 = tq, wq


# ---------------------------------------------------------------------------
# the stage operator
# ---------------------------------------------------------------------------
class Oracle:
    def __init__(self, prob: Problem):
        self.prob = prob
        self.mesh = prob.mesh
        self.el = Element(self.mesh.d, self.mesh.p)
        self.conn = self.mesh.connectivity()
        d = self.mesh.d
        self.nbr = {(k, s): self.mesh.neighbour(k, s) for k in range(d) for s in (-1, 1)}
        self.mult = self.mesh.multiplicity()
        if prob.params.contrib == "q1" and self.mesh.p != 1:
            raise ValueError("the Q1 element contributions are defined for p = 1")
        if not self.mesh.periodic:
            # the subcell bound of Lemma 1 with boundary facets is left open
            # by the paper (Sec. 3.3), and the Q1 form of Sec. 5.3 is stated
            # for the periodic low-order scheme
            if prob.params.flux_mode == "subcell" or prob.params.contrib == "q1":
                raise ValueError("not defined on a non-periodic line")

    # -- global consistent mass matrix, exact solve -------------------------
    @cached_property
    def _mass_lu(self):
        """LU factors of the assembled periodic 1D mass matrices M_k, one per
        axis; M_C = M_1 (x) ... (x) M_d on the tensor-product mesh."""
        p, h = self.mesh.p, self.mesh.h
        G = self.el.t1["mass"]
        out = []
        for k in range(self.mesh.d):
            L = self.mesh.L[k]
            M = np.zeros((L, L))
            for e in range(self.mesh.n[k]):
                idx = [(p * e + a) % L for a in range(p + 1)]
                M[np.ix_(idx, idx)] += h * G
            out.append(scipy.linalg.lu_factor(M))
        return out

    def solve_consistent_mass(self, b):
        """x = M_C^{-1} b for b of shape (m, N): one 1D solve per axis."""
        m = b.shape[0]
        shape = (m,) + tuple(reversed(self.mesh.L))    # axis 0 fastest
        x = b.reshape(shape).copy()
        for k in range(self.mesh.d):
            ax = x.ndim - 1 - k
            xk = np.moveaxis(x, ax, 0)
            flat = xk.reshape(xk.shape[0], -1)
            sol = scipy.linalg.lu_solve(self._mass_lu[k], flat)
            x = np.moveaxis(sol.reshape(xk.shape), 0, ax)
        return np.ascontiguousarray(x).reshape(m, -1)

    def assemble(self, elem_vec):
        """sum over e in E_i of element vectors (m, E, nloc) -> (m, N)."""
        m = elem_vec.shape[0]
        out = np.zeros((m, self.mesh.N))
        for c in range(m):
            np.add.at(out[c], self.conn, elem_vec[c])
        return out

    # -- boundary data of a non-periodic line [KHV §2.1, §3, §4] -----------
    def ghost(self, u, side):
        """Boundary data u_hat at the end side = -1 (lo) or +1 (hi) for the
        interior states u (m, ...): the prescribed state, u itself
        (outflow) or u with reversed momentum (Euler wall)."""
        kind, state = self.prob.bc[0 if side < 0 else 1]
        if kind == "state":
            st = np.asarray(state, dtype=np.float64).reshape((-1,) + (1,) * (u.ndim - 1))
            return np.broadcast_to(st, u.shape).copy()
        out = np.array(u, dtype=np.float64, copy=True)
        if kind == "wall":
            out[1] = -out[1]
        return out

    def llf(self, u_in, u_out, n):
        """Local Lax-Friedrichs flux F(u_L, u_R; n) of [KHV eq. (fluxLLF)]
        on a 1D line: u_L = u_in the interior state, u_R = u_out the
        exterior one, n = +-1 the outward normal, lambda_LR the guaranteed
        speed bound of the Riemann problem along n.  Returns (F, lambda)."""
        F = self.prob.phys
        lam = F.riemann_speed_n(u_in, u_out, np.array([float(n)]))
        return 0.5 * n * (F.flux(u_in)[0] + F.flux(u_out)[0]) - 0.5 * lam * (u_out - u_in), lam

    def boundary_facets(self, U, ue):
        """The two boundary facets of a non-periodic line, per side s = -1
        (lo, element 0, local node 0) and +1 (hi, element n - 1, local node
        p), outward: f^partial = F(u_j, u_hat_j; n) of the end node j (in 1D
        |S| = |c_j| = 1 and phi_j is 1 at the end point), which is also the
        boundary flux of b(phi_i, u_h, u_hat_h) [KHV eqs. (bidef), (aecb)];
        the low-order flux f^L = F(u^e, u_hat^{e'}; n) with u_hat^{e'} the
        boundary data of u^e and its speed lambda_ee'; f_h . n at the end."""
        out = {}
        for s in (-1, 1):
            e = 0 if s < 0 else self.mesh.E - 1
            loc = 0 if s < 0 else self.mesh.p
            uj = U[:, e, loc]
            fb, _ = self.llf(uj, self.ghost(uj, s), s)
            uhe = self.ghost(ue[:, e], s)
            fL, lam = self.llf(ue[:, e], uhe, s)
            out[s] = dict(e=e, loc=loc, node=self.conn[e, loc], fb=fb, fL=fL, lam=float(lam),
                          fhn=s * self.prob.phys.flux(uj)[0], uhat_e=uhe)
        return out

    # -- [KHV §2.2] projected gradient ------------------------------------
    def projected_gradient(self, u):
        """g_h: consistent L2 projection of grad u_h into the CG space,
        (M_C g_k)_i = sum_e int_{K_e} phi_i d_k u_h dx.  Returns (d, m, N)."""
        h, d = self.mesh.h, self.mesh.d
        U = u[:, self.conn]
        g = []
        for k in range(d):
            bk = self.assemble(h ** (d - 1) * np.einsum("ij,cej->cei", self.el.cdiv[k], U))
            g.append(self.solve_consistent_mass(bk))
        return np.stack(g)

    # -- [KHV §2.2] WENO smoothness sensor --------------------------------
    def _deriv_at_gauss(self, T, k, shift_axis=None, shift=0.0):
        """Values of D^k v at the (p+1)^d Gauss points of the reference cell.

        T: coefficient tensors (..., p+1 [axis d-1], ..., p+1 [axis 0]).
        The k_j-th derivative along axis j uses k_j-th forward differences of
        the coefficients times p!/(p-k_j)! and the degree p-k_j basis.  With
        shift_axis set, the polynomial is evaluated at t_q + shift along that
        axis (the neighbour's own coordinates of a point of K_e)."""
        p, d = self.mesh.p, self.mesh.d
        X = T
        # every difference first (exact on nearly equal coefficients), then
        # the evaluation: differencing evaluated values would cancel digits
        for j in range(d):
            if k[j] > 0:
                X = np.diff(X, n=k[j], axis=X.ndim - 1 - j) * float(bz.derivative_factor(p, k[j]))
        for j in range(d):
            ax = X.ndim - 1 - j
            t = self.el.tq + (shift if j == shift_axis else 0.0)
            V = bz.basis_values(p - k[j], t)          # (q, a)
            X = np.moveaxis(np.tensordot(X, V, axes=([ax], [1])), -1, ax)
        return X

    def _gauss_weights_tensor(self):
        d = self.mesh.d
        W = np.ones(())
        for _ in range(d):
            W = np.multiply.outer(W, self.el.wq1)
        return W

    def weno_parts(self, U):
        """Pieces of the WENO sensor of [KHV eqs. (7), (8)] per component:
        beta[c, l, e] = ||u_{h,l}^e||_e^2 of every candidate, omega[c, l, e],
        dev[c, e] = ||u_h^e - u_h^{e,*}||_e, nrm[c, e] = ||u_h^e||_e and the
        sensor gamma[c, e]."""
        prm = self.prob.params
        mesh = self.mesh
        d, p = mesh.d, mesh.p
        m, E = U.shape[0], U.shape[1]
        W = self._gauss_weights_tensor()
        axes_q = tuple(range(-d, 0))
        ks = multi_indices(d, p)
        # candidates: l = 0 own polynomial, then one per facet neighbour
        cands = [(None, None, 0.0)]
        for k in range(d):
            for s in (-1, 1):
                # low neighbour (s=-1) sees a point t of K_e at t + 1
                cands.append((k, self.nbr[(k, s)], -float(s)))
        nl = len(cands)
        wlin = np.array([1.0 - (nl - 1) * prm.w_lin] + [prm.w_lin] * (nl - 1))
        # a boundary facet has no neighbour: its candidate is absent
        present = np.ones((nl, E), dtype=bool)
        for l, (ax, nb, sh) in enumerate(cands):
            if nb is not None:
                present[l] = nb >= 0
        shape = (E,) + (p + 1,) * d
        out = dict(beta=[], omega=[], dev=[], nrm=[], gamma=[])
        for c in range(m):
            T = U[c].reshape(shape)
            vals = []       # vals[l][kk] : (E, q...)
            for (ax, nb, sh) in cands:
                # (an absent candidate is given the element's own polynomial:
                # its weight is zero, so it adds nothing)
                Tl = T if nb is None else T[np.where(nb >= 0, nb, np.arange(E))]
                vals.append([self._deriv_at_gauss(Tl, kk, ax, sh) for kk in ks])
            beta = np.stack([sum(np.sum(W * v ** 2, axis=axes_q) for v in vl)
                             for vl in vals])                 # (nl, E)
            wt = np.where(present, wlin[:, None] / (beta ** (prm.r / 2.0) + prm.eps), 0.0)
            om = wt / wt.sum(axis=0)
            dev2 = 0.0
            for kk in range(len(ks)):
                diff = sum(om[l][(slice(None),) + (None,) * d] * (vals[0][kk] - vals[l][kk])
                           for l in range(1, nl))
                dev2 = dev2 + np.sum(W * diff ** 2, axis=axes_q)
            dev = np.sqrt(np.maximum(dev2, 0.0))
            nrm = np.sqrt(np.maximum(beta[0], 0.0))
            # the ratio of (7) is 0/0 on constant elements; it is regularised
            # with the epsilon of the weights, ||u||_e^2 -> ||u||_e^2 + eps
            ratio = np.minimum(1.0, dev / np.sqrt(np.maximum(beta[0], 0.0) + prm.eps))
            for key, val in (("beta", beta), ("omega", om), ("dev", dev), ("nrm", nrm),
                             ("gamma", 1.0 - ratio ** prm.q)):
                out[key].append(val)
        return {k: np.stack(v) for k, v in out.items()}

    def weno_gamma(self, U):
        """gamma_e of [KHV eq. (7)]; a system takes the minimum over its
        components.  Shape (E,)."""
        mode = self.prob.params.gamma_mode
        E = U.shape[1]
        if mode == "zero":
            return np.zeros(E)
        if mode == "one":
            return np.ones(E)
        return np.min(self.weno_parts(U)["gamma"], axis=0)

    # -- Appendix A ---------------------------------------------------------
    def subcell_dt(self, U, ue):
        """Subcell bound dt_e^max of Lemma 1 [KHV eq. (37)]: boundary nodes
        i with c_i = int_dK phi_i n ds and lambda_0i the Riemann speed of
        (u_0, u_i) along c_i / |c_i|; u_0 is the mass-weighted mean of the
        interior nodes (s = 1).  Without interior nodes (p = 1) u_0 = u^e,
        s = 2 and m_0 = |K_e| (the weight 1/2 of u_0 in the decomposition
        u^e = (u_0 + sum_i m_i u_i / |K_e|) / 2, with the doubled step)."""
        mesh, el, F = self.mesh, self.el, self.prob.phys
        d, p, h = mesh.d, mesh.p, mesh.h
        vol, area = h ** d, h ** (d - 1)
        idx = mesh.local_index()
        lump1 = el.t1["lump"]
        mloc = vol * el.lump
        bnd = np.any((idx == 0) | (idx == p), axis=1)
        cvec = np.zeros((d, mesh.nloc))
        for k in range(d):
            w = area * np.prod([lump1[idx[:, j]] for j in range(d) if j != k], axis=0) if d > 1 \
                else np.ones(mesh.nloc)
            cvec[k] = np.where(idx[:, k] == p, w, 0.0) - np.where(idx[:, k] == 0, w, 0.0)
        cabs = np.sqrt(np.sum(cvec ** 2, axis=0))
        if np.any(~bnd):
            m0 = mloc[~bnd].sum()
            u0 = np.einsum("i,cei->ce", mloc[~bnd], U[:, :, ~bnd]) / m0
            s = 1.0
        else:
            m0, u0, s = vol, ue, 2.0
        bi = np.nonzero(bnd)[0]
        lam = np.stack([F.riemann_speed_n(u0, U[:, :, i], cvec[:, i] / cabs[i]) for i in bi], axis=-1)
        with np.errstate(divide="ignore"):
            t_node = np.min(mloc[bi][None, :] / (cabs[bi][None, :] * lam), axis=-1)
            t_mean = m0 / np.sum(cabs[bi][None, :] * lam, axis=-1)
        return np.minimum(t_node, t_mean) / s

    def shrunk_dt(self, ue, fH_sum, dt_cell):
        """The Remark after [KHV eq. (40)]: start from dt_e of (40) and take
        the largest dt_e <= it with ubar^e = u^e - dt_e |dK|/|K| sum f^H
        admissible (global bounds; Euler: Appendix A with its margin)."""
        h, d = self.mesh.h, self.mesh.d
        D = h ** (d - 1) / h ** d * fH_sum             # ubar(dt) = ue - dt D
        if self.prob.kind == "euler":
            return self._euler_alpha(ue, -dt_cell[None, :] * D, 1.0) * dt_cell
        u, D0 = ue[0], D[0]
        with np.errstate(divide="ignore", invalid="ignore"):
            lim = np.where(D0 > 0, (u - self.prob.u_min) / D0,
                           np.where(D0 < 0, (self.prob.u_max - u) / -D0, np.inf))
        return np.minimum(dt_cell, np.maximum(lim, 0.0))

    def _euler_alpha(self, ubar, f, mi):
        """Largest alpha_i in [0,1] with ubar + alpha f/m_i admissible
        (density, then pressure via P_i(alpha) >= alpha R_i), strict margin
        eps_pos.  ubar, f: (m, ...); returns (...)."""
        eps = self.prob.params.eps_pos
        d = self.mesh.d
        rho, mom, en = ubar[0], ubar[1:1 + d], ubar[-1]
        fr, fm, fe = f[0], f[1:1 + d], f[-1]
        with np.errstate(divide="ignore", invalid="ignore"):
            cond = mi * rho * (1.0 - eps) + fr < 0.0
            a_rho = np.where(cond, (1.0 - eps) * (-mi * rho / np.where(fr == 0, 1, fr)), 1.0)
            Q = mi * (0.5 * np.sum(mom ** 2, axis=0) - rho * en)
            R = (rho * fe + en * fr - np.sum(mom * fm, axis=0)
                 + np.minimum(0.0, fe * fr - 0.5 * np.sum(fm ** 2, axis=0)) / mi)
            condp = R < (1.0 - eps) * Q
            a_p = np.where(condp, (1.0 - eps) * Q / np.where(condp, R, 1.0), 1.0)
        return np.minimum(np.minimum(a_rho, a_p), 1.0)

    # -- one forward-Euler stage ------------------------------------------
    def fe_stage(self, u, dt):
        """u^SSP = forward-Euler stage of [KHV eq. (49)] with the limited
        intermediate states.  u: (m, N).  Returns (u_fe, taps)."""
        prob, prm, mesh, el = self.prob, self.prob.params, self.mesh, self.el
        d, p, h = mesh.d, mesh.p, mesh.h
        F = prob.phys
        vol, area = h ** d, h ** (d - 1)
        nloc = mesh.nloc
        mloc = vol * el.lump                       # m_i^e = int phi_i = |K|/|N_e|
        conn = self.conn
        U = u[:, conn]                             # (m, E, nloc)
        m, E = U.shape[0], U.shape[1]

        # old cell averages [KHV eq. (21)]
        ue = np.einsum("i,cei->ce", mloc, U) / vol

        # ---- step 1: element loop: WENO sensor, stabilisation, residual ---
        g = self.projected_gradient(u)                         # (d, m, N)
        gamma = self.weno_gamma(U)                             # (E,)
        lam_e = np.max(F.node_speed(U), axis=-1)               # (E,)
        nu = lam_e * h / (2.0 * p)                             # [KHV eq. (6)]
        uq = np.einsum("qj,cej->ceq", el.vq, U)
        fq = F.flux(uq)                                        # (d, m, E, q)
        A = area * sum(np.einsum("q,qi,ceq->cei", el.wq, el.dvq[k], fq[k])
                       for k in range(d))                      # int grad phi_i . f(u_h)
        Gn = g[:, :, conn]                                     # (d, m, E, nloc)
        S = nu[None, :, None] * (
            h ** (d - 2) * sum(np.einsum("ij,cej->cei", el.stiff[k], U) for k in range(d))
            - gamma[None, :, None] * area
            * sum(np.einsum("ij,cej->cei", el.cgrad[k], Gn[k]) for k in range(d)))
        r = self.assemble(A - S)      # residual of (10): M_C udot = r (periodic, b = 0)
        bf = None
        if not mesh.periodic:
            # -a(phi_i, u_h) - b(phi_i, u_h, u_hat_h) [KHV eqs. (weak:stab2),
            # (bidef)]: integrating div f(u_h) by parts leaves phi_i f(u_h) . n
            # at the two end points, which b turns into phi_i F(u_h, u_hat_h; n)
            bf = self.boundary_facets(U, ue)
            for sd in (-1, 1):
                r[:, bf[sd]["node"]] -= bf[sd]["fb"]

        # ---- step 2: consistent-mass solve for udot ------------------------
        udot = self.solve_consistent_mass(r)

        # ---- step 3: facet loop -------------------------------------------
        fh_nodes = F.flux(U)                                   # (d, m, E, nloc)
        # canonical facet between element e (low side) and its +e_k neighbour
        fH_c, fL_c, lam_c = [], [], []
        for k in range(d):
            hi = self.nbr[(k, 1)]
            idx = mesh.facet_local_nodes(k, +1)
            # (1/|S|) int_S f_h . n ds, with int_S phi_j ds / |S| = prod lump
            w_face = np.prod([el.t1["lump"][mesh.local_index()[idx, j]]
                              for j in range(d) if j != k], axis=0) if d > 1 else np.ones(1)
            fH_c.append(np.einsum("j,cej->ce", w_face, fh_nodes[k][:, :, idx]))
            lam = F.riemann_speed(ue, ue[:, hi], k)
            fL = 0.5 * (F.flux(ue)[k] + F.flux(ue[:, hi])[k]) - 0.5 * lam * (ue[:, hi] - ue)
            fL_c.append(fL)                                    # [KHV eq. (18)]
            lam_c.append(lam)
        if bf is not None:
            # non-periodic line: the high boundary facet takes the place of
            # the last element's canonical facet (same orientation, +x), with
            # f^H = f^partial and f^L with the boundary data [KHV eqs.
            # (hoflux), (fL)]; the low boundary facet is kept apart (outward)
            eh = bf[1]["e"]
            fH_c[0][:, eh] = bf[1]["fb"]
            fL_c[0][:, eh] = bf[1]["fL"]
            lam_c[0][eh] = bf[1]["lam"]

        def outward(qc, k, s, low=None):
            """facet quantity of element e on side s of axis k, outward; on a
            non-periodic line element 0's low facet takes `low`, the boundary
            facet's own outward value."""
            if s > 0:
                return qc[k]
            v = -qc[k][..., self.nbr[(k, -1)]]
            if bf is not None:
                v = v.copy()
                v[..., 0] = low
            return v

        lo_b = bf[-1] if bf is not None else dict(fb=None, fL=None, lam=None)
        lam_sum = 0.0
        for k in range(d):
            lam_lo = lam_c[k][self.nbr[(k, -1)]]
            if bf is not None:
                lam_lo = lam_lo.copy()
                lam_lo[0] = lo_b["lam"]
            lam_sum = lam_sum + lam_c[k] + lam_lo
        dt_e = vol / (area * lam_sum)                          # [KHV eq. (40)]
        fH_sum = sum(outward(fH_c, k, s, lo_b["fb"]) for k in range(d) for s in (-1, 1))
        if prm.flux_mode == "subcell":
            dt_e = self.subcell_dt(U, ue)                      # [KHV eq. (37)]
        elif prm.flux_mode == "shrink":
            dt_e = self.shrunk_dt(ue, fH_sum, dt_e)            # Remark after (40)
        fL_sum = sum(outward(fL_c, k, s, lo_b["fL"]) for k in range(d) for s in (-1, 1))
        ubarL = ue - dt_e / vol * area * fL_sum                # [KHV eq. (51)]

        # bounds of the scalar limiters per element (Sec. 4.1, 4.2): global,
        # or the range of the cell averages of K_e and its facet neighbours
        # (the low-order average ubar^{e,L} lies in it: it is a convex
        # combination of u^e and the bar states of its facets)
        if prob.kind != "euler" and prm.bounds == "local":
            b_lo, b_hi = ue[0].copy(), ue[0].copy()
            for k in range(d):
                for s_ in (-1, 1):
                    nb = self.nbr[(k, s_)]
                    v = ue[0][nb]
                    if bf is not None:
                        # across a boundary facet: the boundary data u_hat^{e'}
                        # (the low-order average mixes it in)
                        v = np.where(nb >= 0, v, bf[s_]["uhat_e"][0])
                    b_lo = np.minimum(b_lo, v)
                    b_hi = np.maximum(b_hi, v)
        else:
            b_lo, b_hi = np.full(E, prob.u_min), np.full(E, prob.u_max)

        fA_c = [fL_c[k] - fH_c[k] for k in range(d)]           # f^A = f^L - f^H
        phi_e = vol / (2 * d * area)                           # |K_e| / |dK_e|
        fAbar_c = []
        def limit(fA, has_hi, hi, dt_hi=None):
            """limited antidiffusive flux of canonical facets (e, hi) [KHV eq.
            (53) / Appendix A]; where has_hi is False the facet is the
            boundary facet of e, which keeps only e's bounds (e' > E_h)"""
            if prm.alpha_mode == "one":
                return fA
            if prm.alpha_mode == "zero":
                return np.zeros_like(fA)
            if prob.kind == "euler":
                # Appendix A on the pair (u_ee', u_e'e); u_ee' = ubarL_e +
                # alpha |dK_e| dt_e f^A / |K_e| and the mirror for e'
                de = fA / phi_e * dt_e
                dh = -fA / phi_e * dt_e[hi]
                a1 = self._euler_alpha(ubarL, de, 1.0)
                a2 = np.where(has_hi, self._euler_alpha(ubarL[:, hi], dh, 1.0), 1.0)
                return np.minimum(a1, a2)[None] * fA
            # [KHV eq. (53)]: e keeps ubar^e <= its upper bound, e' keeps
            # ubar^{e'} >= its lower bound (and the mirror for f^min)
            with np.errstate(invalid="ignore"):
                fmax = np.minimum(phi_e * (b_hi - ubarL) / dt_e,
                                  np.where(has_hi, phi_e * (ubarL[:, hi] - b_lo[hi]) / dt_e[hi], np.inf))
                fmin = np.maximum(phi_e * (b_lo - ubarL) / dt_e,
                                  np.where(has_hi, phi_e * (ubarL[:, hi] - b_hi[hi]) / dt_e[hi], -np.inf))
            return np.where(fA >= 0.0, np.minimum(fA, fmax), np.maximum(fA, fmin))

        for k in range(d):
            hi = self.nbr[(k, 1)]
            fAbar_c.append(limit(fA_c[k], hi >= 0, hi))
        fAbar_low = None
        if bf is not None:
            # the low boundary facet of element 0, outward: the same one-sided
            # limiter seen from element 0 (a 1-element view of limit())
            fA_lo = lo_b["fL"] - lo_b["fb"]
            if prm.alpha_mode == "one":
                fAbar_low = fA_lo
            elif prm.alpha_mode == "zero":
                fAbar_low = np.zeros_like(fA_lo)
            elif prob.kind == "euler":
                fAbar_low = self._euler_alpha(ubarL[:, 0], fA_lo / phi_e * dt_e[0], 1.0) * fA_lo
            else:
                fmax = phi_e * (b_hi[0] - ubarL[:, 0]) / dt_e[0]
                fmin = phi_e * (b_lo[0] - ubarL[:, 0]) / dt_e[0]
                fAbar_low = np.where(fA_lo >= 0.0, np.minimum(fA_lo, fmax), np.maximum(fA_lo, fmin))

        # ---- step 4: element loop: limited averages, contributions, beta ---
        fAbar_sum = sum(outward(fAbar_c, k, s, fAbar_low) for k in range(d) for s in (-1, 1))
        if prm.flux_mode == "limit":
            ubar = ubarL + dt_e / vol * area * fAbar_sum       # [KHV eq. (44)]
        else:
            ubar = ue - dt_e / vol * area * fH_sum             # f_ee' = f^H, Sec. 4.3 step 4

        # antidiffusive element contributions [KHV eq. (45)], g_i^e = 0
        fgrad_h = area * sum(np.einsum("ij,cej->cei", el.cgrad[k], fh_nodes[k])
                             for k in range(d))                # int grad phi_i . f_h
        fdiv_h = area * sum(np.einsum("ij,cej->cei", el.cdiv[k], fh_nodes[k])
                            for k in range(d))                 # int phi_i div f_h
        fdiv_tot = area * sum(np.einsum("j,cej->ce", el.int_dphi[k], fh_nodes[k])
                              for k in range(d))               # int div f_h
        mi = self.assemble(np.broadcast_to(mloc, (1, E, nloc)).copy())[0]
        udot_lo = None
        if prm.contrib == "q1":
            # low-order time derivative [KHV eq. (weak:low1)], periodic (b = 0):
            # m_i udot_i^L = -a_i - s_i, a_i = sum_e (m_i^e/|K_e|) int div f_h,
            # s_i^e = (m_i^e / dt_e)(u_i - u^e) [KHV eq. (rusdiss)]
            lo = (-(mloc / vol)[None, None, :] * fdiv_tot[:, :, None]
                  - mloc[None, None, :] / dt_e[None, :, None] * (U - ue[:, :, None]))
            udot_lo = self.assemble(lo) / mi
            UdL = udot_lo[:, conn]
            consL = vol * np.einsum("ij,cej->cei", el.mass, UdL) - mloc * UdL
            fe = gamma[None, :, None] * (
                mloc * (U - ue[:, :, None])
                - dt_e[None, :, None] * ((fdiv_h - (mloc / vol) * fdiv_tot[:, :, None]) + consL))
        else:
            Ud = udot[:, conn]
            cons = vol * np.einsum("ij,cej->cei", el.mass, Ud) - mloc * Ud
            gb = np.zeros_like(U)
            if bf is not None:
                # g_i^e of [KHV eq. (aecb)] on the two boundary elements: in 1D
                # the facet integrals are point values at the end, so g_i^e =
                # (delta_{i,end} - m_i^e/|K_e|) (F(u_end, u_hat; n) - f_h . n)
                for sd in (-1, 1):
                    jump = bf[sd]["fb"] - bf[sd]["fhn"]
                    w = -mloc / vol
                    w = w.copy()
                    w[bf[sd]["loc"]] += 1.0
                    gb[:, bf[sd]["e"], :] += w[None, :] * jump[:, None]
            fe = (mloc * (U - ue[:, :, None])
                  + dt_e[None, :, None] * ((A - fgrad_h)
                                           - (fdiv_h - (mloc / vol) * fdiv_tot[:, :, None])
                                           - gb - S - cons))

        # slope limiter [KHV eqs. (54), (55)] / Appendix A
        if prm.beta_mode == "one":
            beta = np.ones(E)
        elif prm.beta_mode == "zero":
            beta = np.zeros(E)
        elif prob.kind == "euler":
            a = self._euler_alpha(np.broadcast_to(ubar[:, :, None], fe.shape), fe,
                                  mloc[None, :])
            beta = np.min(a, axis=-1)
        else:
            ub = ubar[0][:, None]
            f0 = fe[0]
            with np.errstate(divide="ignore", invalid="ignore"):
                # ubar lies in the element's bounds up to rounding; a ratio
                # made negative by a rounding excess is taken as 0
                bpos = np.clip(mloc * (b_hi[:, None] - ub) / np.where(f0 > 0, f0, 1.0), 0.0, 1.0)
                bneg = np.clip(mloc * (b_lo[:, None] - ub) / np.where(f0 < 0, f0, 1.0), 0.0, 1.0)
            bi = np.where(f0 > 0, bpos, np.where(f0 < 0, bneg, 1.0))
            beta = np.min(bi, axis=-1)

        ubar_i = ubar[:, :, None] + beta[None, :, None] * fe / mloc    # [KHV eq. (48)]

        # ---- step 5: SSP stage [KHV eq. (49)] -------------------------------
        if not np.all(dt <= dt_e):
            raise CFLViolation(float(dt), float(dt_e.min()))
        ratio = (dt / dt_e)[None, :, None]
        contrib = mloc * ((1.0 - ratio) * U + ratio * ubar_i)
        u_fe = self.assemble(contrib) / mi

        taps = dict(g=g, gamma=gamma, nu=nu, lam_e=lam_e, r=r, udot=udot, ue=ue,
                    fgrad_h=fgrad_h, fH=np.stack(fH_c), fL=np.stack(fL_c), lam_f=np.stack(lam_c),
                    dt_e=dt_e, ubarL=ubarL, fA=np.stack(fA_c), fAbar=np.stack(fAbar_c),
                    b_lo=b_lo, b_hi=b_hi, fdiv_tot=fdiv_tot, udot_lo=udot_lo,
                    fA_low=(lo_b["fL"] - lo_b["fb"]) if bf is not None else None,
                    fAbar_low=fAbar_low,
                    ubar=ubar, fe=fe, beta=beta, A=A, S=S, u_fe=u_fe)
        return u_fe, taps

    # -- bounds policy after a stage ---------------------------------------
    def clamp(self, u):
        """Scalar problems: values outside [u_min, u_max] by at most a few
        ulps of rounding are clamped and counted; larger excursions are
        reported as violations.  Euler: count nonpositive rho or p."""
        prob = self.prob
        # G of Theorem 1 holds rho > 0, p > 0 (Euler) or u in [u_min, u_max];
        # the tests are written so that a NaN is counted as outside G
        if prob.kind == "euler":
            with np.errstate(invalid="ignore", divide="ignore"):
                bad = int(np.sum(~(u[0] > 0)) + np.sum(~(prob.phys.pressure(u) > 0)))
            return u, 0, bad
        tol = prob.params.clamp_ulps * np.finfo(float).eps * max(abs(prob.u_min), abs(prob.u_max))
        hi = (u > prob.u_max) & (u <= prob.u_max + tol)
        lo = (u < prob.u_min) & (u >= prob.u_min - tol)
        bad = int(np.sum(~((u >= prob.u_min - tol) & (u <= prob.u_max + tol))))
        u = np.where(hi, prob.u_max, np.where(lo, prob.u_min, u))
        return u, int(np.sum(hi) + np.sum(lo)), bad

    def max_dt(self, u):
        """min_e dt_e(u) of [KHV eq. (40)] without running a stage (with the
        flux limiter off: of the stage's own dt_e, eq. (37) or the Remark)."""
        if self.prob.params.flux_mode != "limit" or not self.mesh.periodic:
            return float(np.min(self.fe_stage(u, 0.0)[1]["dt_e"]))
        mesh, F = self.mesh, self.prob.phys
        d, h = mesh.d, mesh.h
        U = u[:, self.conn]
        ue = np.einsum("i,cei->ce", h ** d * self.el.lump, U) / h ** d
        lam_sum = 0.0
        for k in range(d):
            hi, lo = self.nbr[(k, 1)], self.nbr[(k, -1)]
            lam = F.riemann_speed(ue, ue[:, hi], k)
            lam_sum = lam_sum + lam + lam[lo]
        return float(np.min(h ** d / (h ** (d - 1) * lam_sum)))

    def ssp_rk3_step(self, u, dt):
        """Shu-Osher SSP-RK3 with the stage operator above [KHV §5]:
        u1 = L(u), u2 = 3/4 u + 1/4 L(u1), u_new = 1/3 u + 2/3 L(u2)."""
        stats = dict(clamped=0, violations=0)

        def post(v):
            v, nc, nb = self.clamp(v)
            stats["clamped"] += nc
            stats["violations"] += nb
            return v

        u1 = post(self.fe_stage(u, dt)[0])
        u2 = post(0.75 * u + 0.25 * self.fe_stage(u1, dt)[0])
        u3 = post(u / 3.0 + (2.0 / 3.0) * self.fe_stage(u2, dt)[0])
        return u3, stats

    def run(self, u, nsteps, dt=None, cfl=0.5):
        """nsteps SSP-RK3 steps; dt None -> adaptive dt = cfl * min_e dt_e."""
        tot = dict(clamped=0, violations=0)
        for _ in range(nsteps):
            step_dt = dt if dt is not None else cfl * self.max_dt(u)
            u, st = self.ssp_rk3_step(u, step_dt)
            for k in tot:
                tot[k] += st[k]
        return u, tot


class CFLViolation(RuntimeError):
    def __init__(self, dt, dtmin):
        super().__init__(f"dt={dt} exceeds min_e dt_e={dtmin} [KHV eq. (23)]")
        self.dt, self.dtmin = dt, dtmin
