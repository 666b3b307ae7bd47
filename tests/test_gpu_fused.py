"""2D Euler: element pass 2 with the fused update (cem_set_fused_update)
against the separate update kernel (the default).  The nodes whose elements
all lie in one pass-2 block are summed in LDS in the update kernel's element
order with the same rounding, so both paths must give bitwise the same
states, counters and time steps; the separate path is the one every other
GPU test compares with the oracle."""
import numpy as np
import pytest

from paper_2509_04673_amd import workloads as W
from parity_util import announce, gpu_for, random_euler_workload

pytestmark = pytest.mark.gpu

CASES = [
    # ragged blocks: element rows shorter and longer than a block, rows that
    # wrap inside a block, the smallest mesh (the x neighbours coincide)
    ("q2_20x7", lambda: random_euler_workload(2, 2, (20, 7))),
    ("q2_70x9", lambda: random_euler_workload(2, 2, (70, 9))),
    ("q3_33x10", lambda: random_euler_workload(2, 3, (33, 10))),
    ("q1_65x4", lambda: random_euler_workload(2, 1, (65, 4))),
    ("q2_2x3", lambda: random_euler_workload(2, 2, (2, 3))),
    ("quadrants_q3_64", lambda: W.euler2d(seed=2, n=64)),
]


def _run(wl, fused, precision, nsteps):
    s = gpu_for(wl, precision=precision)
    s.set_fused_update(fused)
    for _ in range(nsteps):
        s.step(cfl=0.5)
    out = s.download()
    chk = s.check()
    s.close()
    return out, chk


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("label,make", CASES, ids=[c[0] for c in CASES])
def test_fused_update_is_bitwise_the_separate_update(label, make, precision):
    wl = make()
    a, ca = _run(wl, True, precision, 3)
    b, cb = _run(wl, False, precision, 3)
    announce(f"[fused] {label} {precision}: max |fused - separate| {float(np.max(np.abs(a - b))):.1e}")
    assert np.array_equal(a, b)
    for k in ("dt", "min_dt_e", "violations", "clamped", "cfl_violated", "rho_min", "p_min"):
        assert ca[k] == cb[k], (k, ca[k], cb[k])


def test_fused_update_counts_violations_like_the_separate_update():
    # a state with negative pressure at some nodes: the violations of the
    # first stage are counted in pass 2's counter slots and the update's
    wl = random_euler_workload(2, 2, (24, 11))
    u = wl.u0.copy()
    rng = np.random.default_rng(3)
    bad = rng.choice(u.shape[1], 40, replace=False)
    u[-1, bad] = 0.1 * 0.5 * (u[1, bad] ** 2 + u[2, bad] ** 2) / u[0, bad]   # E below the kinetic energy
    res = {}
    for fused in (True, False):
        s = gpu_for(wl)
        s.upload(u)
        s.set_fused_update(fused)
        s.reset_counters()
        s.stage(0, dt=1e-4)
        res[fused] = (s.download(), s.check())
        s.close()
    announce(f"[fused] violations fused {res[True][1]['violations']}, separate {res[False][1]['violations']}")
    assert res[True][1]["violations"] == res[False][1]["violations"] > 0
    assert np.array_equal(res[True][0], res[False][0], equal_nan=True)


def test_fused_update_batch_is_bitwise_the_separate_update():
    from paper_2509_04673_amd import cem
    from test_gpu_batch import _batch_for
    wls = W.euler_batch(seed=8, sizes=[6, 33, 64, 70, 129])
    outs = {}
    for fused in (1, 0):
        b = _batch_for(wls)
        cem.cem_batch_set_fused_update(b.b, fused)
        b.step(cfl=0.5, nsteps=2)
        outs[fused] = b.download(split=False)
        b.close()
    assert np.array_equal(outs[1], outs[0])
