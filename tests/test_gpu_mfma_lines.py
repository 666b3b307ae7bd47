"""The float64 line passes on the matrix cores (projected gradient, Sec.
2.2; consistent-mass solve, Sec. 4.3 step 2): tiles of 16 lines whose
banded line operator runs as chains of 16x16x4 float64 matrix products.

Forced on (cem_set_line_kernels 1) on meshes whose lines are long enough for
the truncated operators, with line counts and lengths that leave ragged
tiles (line counts not a multiple of 16, lengths not a multiple of the
tile), along axes 0, 1 and 2, for p = 1, 2, 3 (p = 3 reads the operator
from LDS, p = 1, 2 keep it in registers): one stage against the oracle,
every intermediate at relative L-infinity 1e-12; a multi-step run within
the oracle's 1-ulp floor; and on a mesh too big for the oracle the matrix
and vector kernels agree to 1e-11 (the rounding of the mass solve)."""
import numpy as np
import pytest

from paper_2509_04673_amd import workloads as W
from parity_util import (announce, compare_stage, gpu_for, random_euler_workload, random_scalar_workload,
                         rel_linf, run_both, run_tol)

pytestmark = pytest.mark.gpu

TOL = 1e-12
MAT = dict(line_kernels=1)

CASES = [
    ("adv2d_q1_64x65", lambda: random_scalar_workload(2, 1, (64, 65)), None),
    ("kpp2d_q2_48x47", lambda: random_scalar_workload(2, 2, (48, 47), kind="kpp"), None),
    ("euler2d_q2_49x46", lambda: random_euler_workload(2, 2, (49, 46)), None),
    ("euler2d_q3_41x43", lambda: random_euler_workload(2, 3, (41, 43)), None),
    ("adv3d_q1_64x3x63", lambda: random_scalar_workload(3, 1, (64, 3, 63)), None),
    ("euler3d_q2_47x3x50", lambda: random_euler_workload(3, 2, (47, 3, 50)), dict(gamma_mode="one")),
]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("label,make,modes", CASES, ids=[c[0] for c in CASES])
def test_matrix_core_lines_stage_parity(label, make, modes):
    wl = make()
    compare_stage(wl, dict(modes or {}, **MAT), label + "-matrix", TOL)


def test_matrix_core_lines_run_parity():
    wl = W.kpp2d(seed=3, n=64)
    err, floor, st, chk = run_both(wl, 10, dt=None, cfl=0.5, modes=MAT)
    assert err <= run_tol(floor), (err, floor)
    assert chk["violations"] == 0


@pytest.mark.timeout(300)
def test_matrix_and_vector_lines_agree_on_a_large_mesh():
    # the 3D blast shape at 64^3 (10.5M DOFs): g, r, udot and the stage
    # result of one stage, matrix against vector kernels (the same operator
    # rows in other summation orders; udot = M_C^{-1} r is defined to about
    # 4 kappa(M_C) eps ~ 2.4e-12 of its size for 3D Q2, kappa ~ 14^3)
    wl = W.euler3d(seed=0, n=64)
    taps = {}
    for mode in (0, 1):
        s = gpu_for(wl, dict(line_kernels=mode))
        s.stage(0, cfl=0.5)
        taps[mode] = {name: s.tap(name) for name in ("g", "udot", "r")}
        taps[mode]["u"] = s.download()
        s.close()
    m = wl.u0.shape[0]
    for name in ("g", "udot", "r", "u"):
        a, b = taps[1][name], taps[0][name]
        err = rel_linf(np.asarray(a).reshape(-1, m, wl.N), np.asarray(b).reshape(-1, m, wl.N))
        announce(f"[mfma] euler3d 64^3 {name}: matrix vs vector rel Linf {err:.1e}")
        assert err <= 1e-11, (name, err)


MIXED_CASES = [
    ("kpp2d_q2_48x47", lambda: random_scalar_workload(2, 2, (48, 47), kind="kpp")),
    ("euler2d_q3_41x43", lambda: random_euler_workload(2, 3, (41, 43))),
    ("adv2d_q1_64x65", lambda: random_scalar_workload(2, 1, (64, 65))),
    ("euler3d_q2_47x3x50", lambda: random_euler_workload(3, 2, (47, 3, 50))),
]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("label,make", MIXED_CASES, ids=[c[0] for c in MIXED_CASES])
def test_matrix_core_lines_mixed_stage(label, make):
    # the mixed form's float line passes on the matrix cores (float products,
    # float accumulation): one stage against the float64 oracle within the
    # mixed-form stage bounds (rel L1 1e-5, rel Linf 5e-5)
    from parity_util import lumped_mass, oracle_for, rel_l1
    wl = make()
    orc = oracle_for(wl)
    dt = 0.5 * orc.max_dt(wl.u0)
    ufe = orc.clamp(orc.fe_stage(wl.u0, dt)[0])[0]
    s = gpu_for(wl, MAT, precision="mixed")
    s.stage(0, dt=dt)
    got = s.download()
    chk = s.check()
    s.close()
    e1, einf = rel_l1(got, ufe, lumped_mass(orc)), rel_linf(got, ufe)
    announce(f"[mfma] {label} mixed: rel L1 {e1:.2e}, rel Linf {einf:.2e}")
    assert e1 <= 1e-5 and einf <= 5e-5, (e1, einf)
    assert chk["violations"] == 0
