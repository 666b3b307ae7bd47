"""Parity of the strided line passes (projected gradient, Sec. 2.2, and the
consistent-mass solve, Sec. 4.3 step 2) in every tile shape the large meshes
launch: runs of P or 2P outputs per thread (re = 1, 2) and tiles of one, two
or four runs per thread (ky = 1, 2, 4), along axis 1 and along axis 2.

One stage against the oracle on meshes big enough for the launch rule to
pick each shape (asserted per case from the rule restated in
parity_util.line_plan): every intermediate at relative L-infinity 1e-12 per
component in float64 on the vector line kernels, and again on the
matrix-core line tiles (which these mesh sizes take by default), and the
mixed form within the stage bounds of the mixed-form tests.  The 3D meshes run with gamma_e forced to 1 (gamma_mode
"one") to keep the oracle's WENO evaluation out of the test's time; the
sensor does not touch the line passes, and every other intermediate is
still compared.  The full-size 2D Q3 quadrant workload (512^2 cells) is one
of the cases: the benchmark's launch configuration for that mesh."""
import pytest

from paper_2509_04673_amd import workloads as W
from parity_util import (announce, compare_stage, gpu_for, line_plan, lumped_mass, oracle_stage,
                         random_euler_workload, rel_l1, rel_linf)

pytestmark = pytest.mark.gpu

TOL = 1e-12
STAGE_L1 = 1e-5
STAGE_LINF = 5e-5

# label, workload, modes, expected {axis: (re, ky)} in float64, in the mixed form
CASES = [
    ("euler2d_q2_512x512", lambda: random_euler_workload(2, 2, (512, 512)), None,
     {1: (2, 2)}, {1: (2, 2)}),
    ("euler2d_q3_512x512_quadrants", lambda: W.euler2d(seed=0), None,
     {1: (2, 1)}, {1: (2, 2)}),
    ("euler3d_q2_40x48x64", lambda: random_euler_workload(3, 2, (40, 48, 64)), dict(gamma_mode="one"),
     {1: (2, 2), 2: (2, 2)}, {1: (2, 2), 2: (2, 2)}),
    ("euler3d_q2_41x41x65", lambda: random_euler_workload(3, 2, (41, 41, 65)), dict(gamma_mode="one"),
     {1: (1, 4), 2: (2, 2)}, {1: (2, 2), 2: (2, 4)}),
]

_cache = {}


def _oracle_stage(label, wl, modes):
    """One oracle stage per case, shared by the float64 and mixed tests."""
    if label not in _cache:
        _cache[label] = oracle_stage(wl, modes)
    return _cache[label]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("label,make,modes,plan64,plan32", CASES, ids=[c[0] for c in CASES])
def test_line_tiles_fp64(label, make, modes, plan64, plan32):
    wl = make()
    got = {ax: line_plan(wl, ax, "fp64") for ax in range(1, wl.d)}
    announce(f"[lines] {label} float64 plan {got}")
    assert got == plan64
    vec = dict(modes or {}, line_kernels=0)
    compare_stage(wl, vec, label + "-vector", TOL, ref=_oracle_stage(label, wl, modes))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("label,make,modes,plan64,plan32", CASES, ids=[c[0] for c in CASES])
def test_line_tiles_fp64_matrix_cores(label, make, modes, plan64, plan32):
    wl = make()
    mat = dict(modes or {}, line_kernels=1)
    compare_stage(wl, mat, label + "-matrix", TOL, ref=_oracle_stage(label, wl, modes))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("label,make,modes,plan64,plan32", CASES, ids=[c[0] for c in CASES])
def test_line_tiles_mixed(label, make, modes, plan64, plan32):
    wl = make()
    got = {ax: line_plan(wl, ax, "mixed") for ax in range(1, wl.d)}
    announce(f"[lines] {label} mixed plan {got}")
    assert got == plan32
    orc, dt, ufe, taps = _oracle_stage(label, wl, modes)
    s = gpu_for(wl, modes, precision="mixed")
    s.stage(0, dt=dt)
    out = s.download()
    g, udot = s.tap("g"), s.tap("udot")
    chk = s.check()
    s.close()
    mass = lumped_mass(orc)
    e1, einf = rel_l1(out, ufe, mass), rel_linf(out, ufe)
    eg = rel_linf(g.reshape(taps["g"].shape), taps["g"])
    eu = rel_linf(udot.reshape(taps["udot"].shape), taps["udot"])
    announce(f"[lines] {label} mixed: stage rel L1 {e1:.2e}, rel Linf {einf:.2e}; "
             f"g {eg:.2e}, udot {eu:.2e} (float line operators)")
    assert e1 <= STAGE_L1 and einf <= STAGE_LINF, (e1, einf)
    # float line operators: rows cut below 1e-9 of their peak, float rounding
    # amplified by the condition number of M_C (~14^d for p = 2, ~51^d for p = 3)
    assert eg <= 1e-4 and eu <= 1e-4, (eg, eu)
    assert chk["violations"] == 0 and chk["rho_min"] > 0 and chk["p_min"] > 0
