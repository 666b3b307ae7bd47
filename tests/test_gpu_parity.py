"""Parity of the HIP stage (through the C ABI) with the float64 oracle.

Tolerance: relative L-infinity 1e-12 per intermediate and per state after
one stage, and after the stated number of SSP-RK3 steps."""
import numpy as np
import pytest

from paper_2509_04673_amd import workloads as W
from parity_util import (compare_stage, gpu_for, oracle_for, random_euler_workload,
                         random_scalar_workload, run_both, run_tol)

pytestmark = pytest.mark.gpu

TOL = 1e-12

STAGE_CASES = [
    ("adv1d_p2", lambda: random_scalar_workload(1, 2, (37,))),
    ("adv1d_p3", lambda: random_scalar_workload(1, 3, (23,))),
    ("adv2d_q1", lambda: random_scalar_workload(2, 1, (16, 15))),
    ("adv2d_q3", lambda: random_scalar_workload(2, 3, (9, 7))),
    ("kpp2d_q2", lambda: random_scalar_workload(2, 2, (13, 11), kind="kpp")),
    ("adv3d_q2", lambda: random_scalar_workload(3, 2, (5, 4, 6))),
    ("euler1d_p2", lambda: random_euler_workload(1, 2, (29,))),
    ("euler2d_q2", lambda: random_euler_workload(2, 2, (12, 7))),
    ("euler2d_q3", lambda: random_euler_workload(2, 3, (9, 10))),
    ("euler3d_q2", lambda: random_euler_workload(3, 2, (5, 6, 4))),
    ("euler3d_q1", lambda: random_euler_workload(3, 1, (7, 5, 6))),
    # lines long enough for the register-blocked line kernel (p = 1, 2, 3)
    ("adv2d_q1_long", lambda: random_scalar_workload(2, 1, (81, 80))),
    ("kpp2d_q2_long", lambda: random_scalar_workload(2, 2, (64, 63), kind="kpp")),
    ("euler2d_q3_long", lambda: random_euler_workload(2, 3, (55, 54))),
    ("euler3d_q2_mixed", lambda: random_euler_workload(3, 2, (63, 5, 4))),
    ("adv3d_q2_ylong", lambda: random_scalar_workload(3, 2, (4, 63, 5))),
    ("adv3d_q2_zlong", lambda: random_scalar_workload(3, 2, (5, 4, 63))),
]

def _compare_stage(wl, modes=None, label=""):
    return compare_stage(wl, modes, label, TOL)[0]


@pytest.mark.parametrize("label,make", STAGE_CASES, ids=[c[0] for c in STAGE_CASES])
def test_stage_parity(label, make):
    _compare_stage(make(), label=label)


@pytest.mark.parametrize("modes", [dict(gamma_mode="zero", alpha_mode="zero", beta_mode="zero"),
                                   dict(alpha_mode="one", beta_mode="one"),
                                   dict(gamma_mode="one", beta_mode="one")],
                         ids=["LO", "target", "HO"])
def test_stage_parity_method_switches(modes):
    _compare_stage(random_scalar_workload(2, 2, (10, 9), kind="kpp"), modes, "switch")
    _compare_stage(random_euler_workload(2, 2, (8, 9)), modes, "switch-euler")
    _compare_stage(random_euler_workload(3, 2, (4, 5, 3)), modes, "switch-euler3d")


_run_both = run_both
_tol = run_tol


def test_adv1d_full_run_parity():
    # the 1D advection workload at its full size: 64 P2 cells, 200 steps
    wl = W.adv1d(seed=0)
    err, floor, st, chk = _run_both(wl, wl.nsteps, dt=wl.dt)
    assert err <= 1e-12
    assert chk["violations"] == 0 and st["violations"] == 0


def test_kpp2d_small_run_parity():
    wl = W.kpp2d(seed=2, n=16)
    err, floor, st, chk = _run_both(wl, 30, dt=2e-3)
    assert err <= _tol(floor)
    assert chk["violations"] == 0


def test_euler2d_small_run_parity():
    wl = W.euler2d(seed=1, n=12)
    err, floor, st, chk = _run_both(wl, 10, dt=None, cfl=0.5)
    assert err <= _tol(floor)
    assert chk["rho_min"] > 0 and chk["p_min"] > 0


def test_euler3d_small_run_parity():
    wl = W.euler3d(seed=0, n=6)
    err, floor, st, chk = _run_both(wl, 4, dt=None, cfl=0.5)
    assert err <= _tol(floor)
    assert chk["rho_min"] > 0 and chk["p_min"] > 0
    # the counters share the workspace with the per-block dt_e minima: a
    # block count past their capacity would show up here
    assert chk["violations"] == 0 and chk["clamped"] == 0 and chk["cfl_violated"] == 0


def test_kpp2d_full_size_stage_parity():
    # the KPP workload at its full size (256^2 Q2) in the benchmark's launch
    # configuration: one stage, every intermediate
    _compare_stage(W.kpp2d(seed=0), label="kpp2d-full")


def test_graph_replay_matches_direct_launches():
    # cem_step replays a captured HIP graph; every replay, with downloads and
    # other eager work in between, must equal the directly launched stages
    from paper_2509_04673_amd import cem
    wl = W.kpp2d(seed=4, n=64)
    a = gpu_for(wl)
    b = gpu_for(wl)
    cem.cem_set_graphs(b.ctx, 0)
    for step in range(5):
        a.step(dt=2e-3)
        b.step(dt=2e-3)
        ua, ub = a.download(), b.download()
        assert np.array_equal(ua, ub), step
    ca, cb = a.check(), b.check()
    assert ca["dt"] == cb["dt"] == 2e-3 and ca["violations"] == 0
    a.close()
    b.close()


def test_adaptive_dt_and_cfl_flag():
    # stage 0 picks dt = cfl * min_e dt_e; a fixed dt above min_e dt_e raises
    # the CFL flag (CEM_ECFL) through the invariant check
    wl = W.euler2d(seed=3, n=16)
    orc = oracle_for(wl)
    s = gpu_for(wl)
    s.step(cfl=0.5)
    chk = s.check()
    assert abs(chk["dt"] - 0.5 * orc.max_dt(wl.u0)) <= 1e-14 * chk["dt"]
    assert chk["cfl_violated"] == 0
    s.upload(wl.u0)
    s.step(dt=4.0 * orc.max_dt(wl.u0))
    chk = s.check()
    # the flag is set; the status is CEM_ECFL, or CEM_EIDP (reported ahead of
    # it) when the oversized step also left the invariant domain
    assert chk["cfl_violated"] == 1
    assert (chk["status"] == -4 and chk["violations"] == 0) or \
        (chk["status"] == -5 and chk["violations"] > 0), chk
    s.close()
