"""Design-order pin of the oracle against the paper's printed convergence
table (Section 5.1.1, Table 1; fixture tests/golden/eoc_advection.txt)."""
import os

import numpy as np
import pytest

from oracle import Mesh, Oracle, Params, Problem
from oracle import bernstein as bz

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "eoc_advection.txt")


def _golden():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    return {int(r[0]): dict(p1=float(r[1]), p1l=float(r[2]), p2=float(r[3]), p2l=float(r[4]))
            for r in rows}


def _gauss_profile(x):
    return np.exp(-100.0 * (x - 0.5) ** 2)


def _run(p, n, target, dt_over_h):
    mesh = Mesh(1, p, (n,), (0.0,), (1.0,))
    prm = Params(w_lin=1e-3)
    if target:
        prm.alpha_mode = prm.beta_mode = "one"
    prob = Problem(mesh, "advection", (1.0,), params=prm)
    orc = Oracle(prob)
    # L2 projection of u0 ([KHV §5.1.1]) with a 12-point rule per cell
    t, w = bz.gauss(12)
    B = bz.basis_values(p, t)
    b = np.zeros(mesh.N)
    for e in range(n):
        np.add.at(b, orc.conn[e], mesh.h * (B.T @ (w * _gauss_profile(mesh.h * (e + t)))))
    u = orc.solve_consistent_mass(b[None])
    # global bounds from the initial Bernstein coefficients (limited run)
    prob.u_min, prob.u_max = (-np.inf, np.inf) if target else (float(u.min()), float(u.max()))
    nst = int(round(1.0 / (dt_over_h * mesh.h)))
    u, st = orc.run(u, nst, dt=1.0 / nst)
    assert st["violations"] == 0
    err = 0.0
    for e in range(n):
        uh = B @ u[0, orc.conn[e]]
        err += mesh.h * np.sum(w * (uh - _gauss_profile(mesh.h * (e + t))) ** 2)
    return np.sqrt(err)


# time step: half of the subcell IDP bound of Lemma 1 (eq. 37) for the
# unlimited average: h/6 for P2 (s = 1), h/4 for P1 (s = 2)
def test_p2_target_matches_printed_errors():
    gold = _golden()
    errs = {n: _run(2, n, True, 0.5 / 6.0) for n in (32, 64, 128)}
    for n in (64, 128):
        # our reading of the unspecified details reproduces the printed
        # target errors to a few percent on the resolved meshes
        assert abs(errs[n] / gold[n]["p2"] - 1.0) < 0.1, (n, errs[n], gold[n]["p2"])
    eoc = np.log2(errs[64] / errs[128])
    assert 2.8 < eoc < 3.2


def test_p2_limited_rate_matches_printed_rate():
    gold = _golden()
    errs = {n: _run(2, n, False, 0.5 / 6.0) for n in (32, 64, 128)}
    for a, b in ((32, 64), (64, 128)):
        ours = np.log2(errs[a] / errs[b])
        paper = np.log2(gold[a]["p2l"] / gold[b]["p2l"])
        assert abs(ours - paper) < 0.15, (a, b, ours, paper)
    # global bounds on Bernstein coefficients cost accuracy (peak clipping)
    assert all(errs[n] / gold[n]["p2l"] < 3.0 for n in errs)


def test_p1_target_is_at_least_second_order():
    errs = [_run(1, n, True, 0.5 / 4.0) for n in (64, 128)]
    assert np.log2(errs[0] / errs[1]) > 1.9
