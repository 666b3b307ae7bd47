"""The Q1 element contributions of Sec. 5.3 (cem_params.contrib =
CEM_CONTRIB_Q1) on the GPU against the oracle: scalar problems, p = 1,
float64, with the low-order time derivative of Sec. 3 in the udot tap.

Tolerances: one stage, relative L-infinity 1e-12 per intermediate (udot
against the oracle's low-order derivative) and for the stage result; runs
within the oracle's own 1-ulp sensitivity floor.  The paper's 2D setting
(flux limiter off through alpha = 1, dt_e of eq. 40, fixed dt) is one of
the cases."""
import numpy as np
import pytest

from paper_2509_04673_amd import workloads as W
from parity_util import compare_stage, gpu_for, random_euler_workload, random_scalar_workload, run_both, run_tol

pytestmark = pytest.mark.gpu

TOL = 1e-12
Q1 = dict(contrib="q1")

CASES = [
    ("adv1d_p1", lambda: random_scalar_workload(1, 1, (41,))),
    ("adv2d_q1", lambda: random_scalar_workload(2, 1, (13, 11))),
    ("kpp2d_q1", lambda: random_scalar_workload(2, 1, (16, 15), kind="kpp")),
    ("kpp2d_q1_2x2", lambda: random_scalar_workload(2, 1, (2, 2), kind="kpp")),
    ("adv3d_q1", lambda: random_scalar_workload(3, 1, (5, 4, 6))),
]

MODES = [
    ("method", {}),
    ("flux_limiter_off", dict(alpha_mode="one")),          # the paper's 2D runs
    ("target", dict(alpha_mode="one", beta_mode="one", gamma_mode="one")),
    ("local_bounds", dict(bounds="local")),
    ("subcell", dict(flux_mode="subcell")),
]


@pytest.mark.parametrize("mlabel,modes", MODES, ids=[m[0] for m in MODES])
@pytest.mark.parametrize("label,make", CASES, ids=[c[0] for c in CASES])
def test_q1_contributions_stage_parity(label, make, mlabel, modes):
    wl = make()
    floors = None
    if min(wl.n) == 2:
        # two cells per axis with p = 1: the periodic gradient operator is
        # zero, g is rounding noise on both sides
        floors = {"g": float(np.max(np.abs(wl.u0))) * wl.n[0] / (wl.hi[0] - wl.lo[0])}
    compare_stage(wl, dict(Q1, **modes), f"{label}-q1-{mlabel}", TOL, floors=floors)


def test_q1_kpp_run_in_the_papers_setting():
    # Sec. 5.3.2's KPP problem on Q1 with the flux limiter off (alpha = 1),
    # dt_e of eq. (40) and a fixed global time step, WENO-L (gamma_e and
    # beta_e active), 20 steps
    wl = W.kpp2d(seed=1, n=32, p=1)
    err, floor, st, chk = run_both(wl, 20, dt=2e-3, modes=dict(Q1, alpha_mode="one"))
    assert err <= run_tol(floor), (err, floor)
    assert chk["violations"] == 0 and st["violations"] == 0
    assert chk["u_min"][0] >= wl.u0.min() and chk["u_max"][0] <= wl.u0.max()


@pytest.mark.parametrize("bad", ["degree", "euler", "mixed", "batch"])
def test_q1_contributions_rejected_outside_their_scope(bad):
    from paper_2509_04673_amd.cem import BatchSolver, CemError
    with pytest.raises(CemError):
        if bad == "degree":
            gpu_for(random_scalar_workload(2, 2, (4, 4)), Q1)
        elif bad == "euler":
            gpu_for(random_euler_workload(2, 1, (4, 4)), Q1)
        elif bad == "mixed":
            gpu_for(random_scalar_workload(2, 1, (4, 4)), Q1, precision="mixed")
        else:
            w = random_scalar_workload(2, 1, (4, 4))
            BatchSolver([(w.d, w.p, w.n, w.lo, w.hi)], w.kind, w.velocity, contrib="q1")
