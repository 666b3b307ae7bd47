"""Local bounds of the scalar limiters (Sec. 4.1, 4.2 admit local or global
ones): per element, the range of the stage input's cell averages of K_e and
its facet neighbours, imposed on the flux-limited average (eq. 53) and on
the element's slope-limited states (eq. 55).

Tolerances: one stage, relative L-infinity 1e-12 per intermediate (the
bounds themselves included) and for the stage result; runs within the
oracle's own 1-ulp sensitivity floor; batched problems match single ones to
1e-12 (float64) or 1e-6 (mixed form: float rounding in other orders)."""
import numpy as np
import pytest

from paper_2509_04673_amd import workloads as W
from parity_util import (announce, compare_stage, gpu_for, random_scalar_workload, rel_linf, run_both,
                         run_tol)

pytestmark = pytest.mark.gpu

TOL = 1e-12
LOCAL = dict(bounds="local")

CASES = [
    ("adv1d_p1", lambda: random_scalar_workload(1, 1, (41,))),
    ("adv1d_p3", lambda: random_scalar_workload(1, 3, (23,))),
    ("adv2d_q1", lambda: random_scalar_workload(2, 1, (16, 15))),
    ("adv2d_q2", lambda: random_scalar_workload(2, 2, (13, 11))),
    ("adv2d_q3", lambda: random_scalar_workload(2, 3, (9, 7))),
    ("kpp2d_q2", lambda: random_scalar_workload(2, 2, (13, 11), kind="kpp")),
    ("kpp2d_q3_long", lambda: random_scalar_workload(2, 3, (48, 9), kind="kpp")),
    ("kpp2d_q2_2x2", lambda: random_scalar_workload(2, 2, (2, 2), kind="kpp")),
    ("adv3d_q1", lambda: random_scalar_workload(3, 1, (6, 5, 4))),
    ("adv3d_q2", lambda: random_scalar_workload(3, 2, (5, 4, 6))),
]


@pytest.mark.parametrize("label,make", CASES, ids=[c[0] for c in CASES])
def test_local_bounds_stage_parity(label, make):
    wl = make()
    floors = None
    if min(wl.n) == 2:
        # two cells per axis: the p-independent parts of g cancel to
        # rounding (see the edge-case tests)
        floors = {"g": float(np.max(np.abs(wl.u0))) * wl.n[0] / (wl.hi[0] - wl.lo[0])}
    errs, taps = compare_stage(wl, LOCAL, f"{label}-local", TOL, floors=floors)
    lo, hi = taps["b_lo"], taps["b_hi"]
    tol = 1e-12 * float(np.max(np.abs(wl.u0)))
    assert np.all(taps["ubar"][0] >= lo - tol) and np.all(taps["ubar"][0] <= hi + tol)
    # the local bounds are tighter than the global ones somewhere, so the
    # limiters see a different constraint
    assert np.any(hi < wl.u0.max()) or np.any(lo > wl.u0.min())


def test_local_bounds_limit_more_than_global():
    # on rough advection data (noise, plateaus) the local bounds make both
    # limiters act more than the global ones do (the oracle: 315 against 170
    # slope-limited elements)
    wl = random_scalar_workload(2, 2, (20, 17), seed=3)
    res = {}
    for mode in ("global", "local"):
        s = gpu_for(wl, dict(bounds=mode))
        s.stage(0, dt=2e-3)
        res[mode] = (s.tap("beta"), s.tap("ubar"), s.tap("ubarL"))
        s.close()
    nb = {m: int(np.sum(r[0] < 0.999)) for m, r in res.items()}
    announce(f"[bounds] slope-limited elements (beta < 0.999): global {nb['global']}, local {nb['local']}")
    assert nb["local"] > nb["global"] > 0
    # the flux-limited averages differ from the low-order ones by the
    # limited fluxes: the local bounds take more of f^A away
    dg = np.abs(res["global"][1] - res["global"][2]).sum()
    dl = np.abs(res["local"][1] - res["local"][2]).sum()
    announce(f"[bounds] sum |ubar - ubarL|: global {dg:.3e}, local {dl:.3e}")
    assert dl < dg


RUNS = [
    ("kpp2d_q2_24", lambda: W.kpp2d(seed=1, n=24), 12, None),
    ("adv2d_q3_rand", lambda: random_scalar_workload(2, 3, (12, 10), seed=5), 8, 2e-3),
    ("adv3d_q2_rand", lambda: random_scalar_workload(3, 2, (6, 5, 6), seed=2), 4, 2e-3),
]


@pytest.mark.parametrize("label,make,nsteps,dt", RUNS, ids=[r[0] for r in RUNS])
def test_local_bounds_run_parity(label, make, nsteps, dt):
    wl = make()
    err, floor, st, chk = run_both(wl, nsteps, dt=dt, cfl=0.5, modes=LOCAL)
    assert err <= run_tol(floor), (err, floor)
    assert chk["violations"] == 0 == st["violations"]
    assert chk["u_min"][0] >= wl.u0.min() and chk["u_max"][0] <= wl.u0.max()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_local_bounds_batch_matches_single(precision):
    from test_gpu_batch import _batch_for, _singles
    wls = [random_scalar_workload(2, 2, (n, n + 3), kind="kpp", seed=n) for n in (20, 57, 70)]
    b = _batch_for(wls, precision=precision, bounds="local")
    b.step(dt=1e-3, nsteps=3)
    got = b.download()
    chk = b.check()
    b.close()
    ref = _singles(wls, 3, 1e-3, 0.0, precision=precision, bounds="local")
    for k, (g, r) in enumerate(zip(got, ref)):
        err = rel_linf(np.asarray(g).reshape(1, -1), np.asarray(r).reshape(1, -1))
        announce(f"[bounds] batch {precision} problem {k}: batch vs single rel Linf {err:.1e}")
        # the mixed form's float line passes run with other run lengths in
        # the batched launches (other summation orders): float-sized
        # differences, as for the Euler batch
        assert err <= (TOL if precision == "fp64" else 1e-6), (k, err)
        assert chk[k]["violations"] == 0


def test_bounds_mode_out_of_range_rejected():
    from paper_2509_04673_amd.cem import CemError
    wl = random_scalar_workload(2, 2, (4, 4))
    with pytest.raises(CemError):
        gpu_for(wl, dict(bounds=2))
