"""Parity of the HIP stage with the oracle when the flux limiter is off
(Sec. 4.3, steps 3-4): f_ee' = f^H of eq. (42), with dt_e the subcell bound
of Lemma 1 (eq. 37) or the bound of eq. (40) reduced until the cell average
is admissible (the Remark after eq. 40).

Tolerance: relative L-infinity 1e-12 per intermediate and for the stage
result; runs within the oracle's own 1-ulp sensitivity floor."""
import numpy as np
import pytest

from paper_2509_04673_amd import workloads as W
from parity_util import (compare_stage, gpu_for, random_euler_workload, random_scalar_workload,
                         run_both, run_tol)

pytestmark = pytest.mark.gpu

TOL = 1e-12

CASES = [
    ("adv1d_p1", lambda: random_scalar_workload(1, 1, (41,))),
    ("adv1d_p2", lambda: random_scalar_workload(1, 2, (37,))),
    ("adv2d_q1", lambda: random_scalar_workload(2, 1, (16, 15))),
    ("adv2d_q3", lambda: random_scalar_workload(2, 3, (9, 7))),
    ("kpp2d_q2", lambda: random_scalar_workload(2, 2, (13, 11), kind="kpp")),
    ("kpp2d_q2_long", lambda: random_scalar_workload(2, 2, (64, 63), kind="kpp")),
    ("adv3d_q2", lambda: random_scalar_workload(3, 2, (5, 4, 6))),
    ("euler1d_p2", lambda: random_euler_workload(1, 2, (29,))),
    ("euler2d_q1", lambda: random_euler_workload(2, 1, (12, 11))),
    ("euler2d_q2", lambda: random_euler_workload(2, 2, (12, 7))),
    ("euler2d_q3", lambda: random_euler_workload(2, 3, (9, 10))),
    ("euler3d_q1", lambda: random_euler_workload(3, 1, (7, 5, 6))),
    ("euler3d_q2", lambda: random_euler_workload(3, 2, (5, 6, 4))),
]


@pytest.mark.parametrize("mode", ["subcell", "shrink"])
@pytest.mark.parametrize("label,make", CASES, ids=[c[0] for c in CASES])
def test_flux_off_stage_parity(label, make, mode):
    wl = make()
    errs, taps = compare_stage(wl, dict(flux_mode=mode), f"{label}-{mode}", TOL)
    # the intermediate averages are admissible (Lemma 1; the Remark)
    ubar = taps["ubar"]
    assert np.all(taps["dt_e"] > 0.0)
    if wl.kind == "euler":
        assert np.all(ubar[0] > 0.0)
    else:
        assert ubar.min() >= wl.u0.min() - 1e-12 and ubar.max() <= wl.u0.max() + 1e-12


def test_kpp2d_subcell_run_parity():
    wl = W.kpp2d(seed=2, n=16)
    err, floor, st, chk = run_both(wl, 20, dt=None, cfl=0.5, modes=dict(flux_mode="subcell"))
    assert err <= run_tol(floor)
    assert chk["violations"] == 0 and chk["cfl_violated"] == 0


def test_euler2d_shrink_run_parity():
    wl = W.euler2d(seed=1, n=12)
    err, floor, st, chk = run_both(wl, 10, dt=None, cfl=0.5, modes=dict(flux_mode="shrink"))
    assert err <= run_tol(floor)
    assert chk["rho_min"] > 0 and chk["p_min"] > 0


def test_euler3d_subcell_run_parity():
    wl = W.euler3d(seed=0, n=6)
    err, floor, st, chk = run_both(wl, 3, dt=None, cfl=0.5, modes=dict(flux_mode="subcell"))
    assert err <= run_tol(floor)
    assert chk["rho_min"] > 0 and chk["p_min"] > 0


def test_flux_mode_out_of_range_rejected():
    from paper_2509_04673_amd.cem import CemError
    wl = random_euler_workload(2, 2, (4, 4))
    with pytest.raises(CemError):
        gpu_for(wl, dict(flux_mode=3))
