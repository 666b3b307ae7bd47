"""The invariant-domain checks of the library fire, and count what the
oracle counts (Theorem 1, Sec. 3.3: the limited stage keeps every state in
G; G is [u_min, u_max] for scalar problems with global bounds, Sec. 4.1-4.2,
and rho > 0, p > 0 for the Euler equations, Sec. 5.2 and Appendix A).

All conditions are forced from the host: inadmissible or non-finite states
are uploaded, or a limiter is switched off through the method switches.
Every kernel runs to its normal end; only the counters and the returned
status are checked.  Also: the global time step taken from a block-reduced
min_e dt_e on a mesh whose last tile row is partly past the mesh edge (the
element pass's exchange barrier then runs in waves that mix live lanes and
lanes past the edge)."""
import math

import numpy as np
import pytest

from oracle import Mesh, Oracle, Params, Problem
from paper_2509_04673_amd import workloads as W
from paper_2509_04673_amd.cem import CemError
from parity_util import announce, gpu_for, oracle_for, random_scalar_workload

pytestmark = pytest.mark.gpu

EIDP, ECFL = -5, -4


def _pressure(u, g=1.4):
    d = u.shape[0] - 2
    return (g - 1.0) * (u[-1] - 0.5 * np.sum(u[1:1 + d] ** 2, axis=0) / u[0])


def test_scalar_state_outside_bounds():
    wl = W.kpp2d(seed=0, n=12)
    lo, hi = float(wl.u0.min()), float(wl.u0.max())
    u = wl.u0.copy()
    u[0, [5, 77, 300]] = hi + 1.0
    u[0, [11, 400]] = lo - 0.5
    s = gpu_for(wl)                       # bounds from the clean state
    s.upload(u)
    s.set_bounds(lo, hi)
    chk = s.check()
    announce(f"[inv] scalar out of bounds: {chk}")
    assert chk["status"] == EIDP
    assert chk["state_violations"] == 5 and chk["nonfinite"] == 0
    assert chk["violations"] == 0          # no stage has run
    assert chk["u_max"][0] == hi + 1.0 and chk["u_min"][0] == lo - 0.5
    # a value within the round-off clamp width is not a violation
    u2 = wl.u0.copy()
    u2[0, 3] = hi * (1.0 + 8 * np.finfo(float).eps)
    s.upload(u2)
    chk = s.check()
    assert chk["status"] == 0 and chk["state_violations"] == 0, chk
    # NaN: counted as non-finite and as outside G; the extrema show it
    u3 = wl.u0.copy()
    u3[0, 123] = np.nan
    s.upload(u3)
    chk = s.check()
    announce(f"[inv] scalar NaN: {chk}")
    assert chk["status"] == EIDP
    assert chk["nonfinite"] == 1 and chk["state_violations"] == 1
    assert math.isnan(chk["u_min"][0]) and math.isnan(chk["u_max"][0])
    # bounds cannot be taken from a state holding NaN
    with pytest.raises(CemError):
        s.set_bounds()
    s.close()


def test_euler_state_not_admissible():
    wl = W.euler2d(seed=1, n=12)
    u = wl.u0.copy()
    i, j = 50, 401
    # node i: p = -0.04 with rho > 0; node j: rho < 0
    u[3, i] = 0.5 * (u[1, i] ** 2 + u[2, i] ** 2) / u[0, i] - 0.1
    u[0, j] = -abs(u[0, j])
    pr = _pressure(u)
    expect = int(np.sum(~(u[0] > 0)) + np.sum(~(pr > 0)))
    s = gpu_for(wl)
    s.upload(u)
    chk = s.check()
    announce(f"[inv] euler inadmissible: expect {expect}, {chk}")
    assert expect >= 2
    assert chk["status"] == EIDP and chk["state_violations"] == expect
    assert chk["rho_min"] == u[0].min()
    assert chk["p_min"] < 0
    # NaN energy at one node: p is NaN there
    u2 = wl.u0.copy()
    u2[3, 7] = np.nan
    s.upload(u2)
    chk = s.check()
    announce(f"[inv] euler NaN: {chk}")
    assert chk["status"] == EIDP and chk["nonfinite"] == 1 and chk["state_violations"] == 1
    assert chk["rho_min"] > 0 and math.isnan(chk["p_min"])
    s.close()


@pytest.mark.parametrize("modes", [dict(alpha_mode="one", beta_mode="one"),
                                   dict(gamma_mode="one", alpha_mode="one", beta_mode="one")],
                         ids=["target", "HO"])
def test_unlimited_scalar_run_counts_violations_like_the_oracle(modes):
    # with both limiters off the discrete maximum principle fails; every
    # stage result outside [u_min, u_max] beyond round-off is counted, by the
    # library per stage in the update kernel and by the oracle per stage
    wl = W.kpp2d(seed=0, n=12)
    orc = oracle_for(wl, modes)
    dt = 0.5 * orc.max_dt(wl.u0)
    u_ref, st = orc.run(wl.u0.copy(), 2, dt=dt)
    s = gpu_for(wl, modes)
    s.step(dt=dt)
    s.step(dt=dt)
    chk = s.check()
    s.close()
    announce(f"[inv] unlimited KPP {modes}: oracle {st['violations']}, library {chk['violations']}")
    assert st["violations"] > 0
    assert chk["status"] == EIDP
    assert chk["violations"] == st["violations"]


def test_euler_blast_without_slope_limiter_counts_violations_like_the_oracle():
    # a 1e5 pressure jump with the slope limiter off: the first stage whose
    # result leaves rho > 0, p > 0 is reported, with the oracle's count
    mesh = Mesh(1, 2, (24,), (0.0,), (1.0,))
    x = mesh.node_coords()[:, 0]
    pr = np.where(np.abs(x - 0.5) < 0.1, 1000.0, 0.01)
    u0 = np.stack([np.ones_like(x), 0 * x, pr / 0.4])
    wl = W.Workload("blast1d", 1, 2, (24,), (0.0,), (1.0,), "euler", u0)
    orc = Oracle(Problem(mesh, "euler", params=Params(beta_mode="one")))
    s = gpu_for(wl, dict(beta_mode="one"))
    s.set_graphs(False)
    u = u0.copy()
    rk = [(0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0)]
    for step in range(10):
        dt = 0.5 * orc.max_dt(u)
        s.u_base.copy_(s.u)                  # u^n of the step (cem_step does this)
        v = u
        for k, (a, b) in enumerate(rk):
            with np.errstate(invalid="ignore", divide="ignore"):
                v, _, bad = orc.clamp(a * u + b * orc.fe_stage(v, dt)[0])
            s.reset_counters()
            s.stage(k, dt=dt)
            chk = s.check()
            announce(f"[inv] blast step {step} stage {k}: oracle {bad}, library {chk['violations']}")
            assert chk["violations"] == bad
            if bad:
                assert chk["status"] == EIDP
                s.close()
                return
        u = v
    pytest.fail("the unlimited blast never left the admissible set")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("flux_mode", ["limit", "subcell"])
def test_block_reduced_dt_on_a_ragged_tile_row(precision, flux_mode):
    # 32 x 22 cells: the last row of 16 x 8 element tiles holds 6 rows, so
    # its second wave mixes live lanes and lanes past the mesh edge; the
    # adaptive dt = cfl min_e dt_e comes from the per-block minima
    wl = random_scalar_workload(2, 2, (32, 22), kind="kpp")
    modes = dict(flux_mode=flux_mode)
    orc = oracle_for(wl, modes)
    dte = orc.fe_stage(wl.u0, 0.0)[1]["dt_e"]
    s = gpu_for(wl, modes, precision=precision)
    s.stage(0, cfl=0.5)
    got_dte = s.tap("dt_e")
    chk = s.check()
    s.close()
    announce(f"[inv] ragged tile row {precision} {flux_mode}: dt {chk['dt']:.17g} vs "
             f"{0.5 * dte.min():.17g}, min dt_e {chk['min_dt_e']:.17g}")
    assert abs(chk["min_dt_e"] - dte.min()) <= 1e-12 * dte.min()
    assert abs(chk["dt"] - 0.5 * dte.min()) <= 1e-12 * dte.min()
    assert chk["min_dt_e"] == got_dte.min()
