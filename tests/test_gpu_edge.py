"""Edge cases of the HIP stage against the oracle: the smallest meshes the
library accepts (two cells per axis, where the left and right facet
neighbours are the same element and every line is shorter than the line
operators' half-width) and single-cell-thick directions mixed with long
ones.  Tolerance: relative L-infinity 1e-12 per intermediate."""
import numpy as np
import pytest

from parity_util import compare_stage, random_euler_workload, random_scalar_workload

pytestmark = pytest.mark.gpu

CASES = [
    ("adv1d_p1_n2", lambda: random_scalar_workload(1, 1, (2,))),
    ("adv1d_p3_n2", lambda: random_scalar_workload(1, 3, (2,))),
    ("euler1d_p2_n2", lambda: random_euler_workload(1, 2, (2,))),
    ("kpp2d_q2_2x2", lambda: random_scalar_workload(2, 2, (2, 2), kind="kpp")),
    ("adv2d_q3_2x17", lambda: random_scalar_workload(2, 3, (2, 17))),
    ("euler2d_q3_2x3", lambda: random_euler_workload(2, 3, (2, 3))),
    ("euler2d_q1_70x2", lambda: random_euler_workload(2, 1, (70, 2))),
    ("adv3d_q2_2x2x2", lambda: random_scalar_workload(3, 2, (2, 2, 2))),
    ("euler3d_q1_2x2x2", lambda: random_euler_workload(3, 1, (2, 2, 2))),
    ("euler3d_q2_2x3x2", lambda: random_euler_workload(3, 2, (2, 3, 2))),
]


def _floors(wl):
    # with p = 1 and two cells along an axis the periodic gradient operator
    # is exactly zero there (each node's left and right elements cancel), so
    # g is rounding noise on both sides: measure it against |u| / h.  On
    # these meshes the sampled data are symmetric enough that whole
    # quantities vanish up to rounding (the velocities sin(2 pi x / L) of
    # the random Euler data at x = 0 and L / 2; the momentum residual of a
    # pressure that two cells hold symmetrically): the residual, udot, f^A
    # and the stage result are measured against their largest quantity
    h = (wl.hi[0] - wl.lo[0]) / wl.n[0]
    fl = {"g": float(np.max(np.abs(wl.u0))) / h}
    if wl.kind == "euler":
        fl.update(r="whole", udot="whole", fA="whole", u_fe="whole")
    return fl


@pytest.mark.parametrize("label,make", CASES, ids=[c[0] for c in CASES])
def test_smallest_meshes_stage_parity(label, make):
    wl = make()
    compare_stage(wl, label=label, floors=_floors(wl))


@pytest.mark.parametrize("mode", ["subcell", "shrink"])
def test_smallest_meshes_flux_off(mode):
    for wl in (random_scalar_workload(2, 2, (2, 2), kind="kpp"), random_euler_workload(3, 2, (2, 2, 2))):
        compare_stage(wl, dict(flux_mode=mode), f"{wl.kind}-{wl.n}-{mode}", floors=_floors(wl))
