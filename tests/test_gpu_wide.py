"""Parity of the strided line passes with runs of 2P outputs per thread.

Meshes large enough that the axis-1 passes (projected gradient, mass solve)
leave 2048 blocks of 32 lines x 16P outputs take runs of 2P instead of P
(the benchmark's Euler meshes do).  One stage against the oracle, every
intermediate, relative L-infinity 1e-12, for p = 1, 2, 3."""
import math

import pytest

from parity_util import compare_stage, oracle_stage, random_euler_workload, random_scalar_workload

pytestmark = pytest.mark.gpu

TOL = 1e-12

W_HALF = {1: 30, 2: 44, 3: 57}      # float64 line-operator half-widths


def takes_wide_runs(wl):
    """The run-length rule of the strided passes for axis 1, restated."""
    p, m = wl.p, wl.u0.shape[0]
    L0, L1 = p * wl.n[0], p * wl.n[1]
    blocks = math.ceil(m * L0 / 32) * math.ceil(L1 / (16 * p))
    return L1 >= 2 * p + 2 * W_HALF[p] and blocks >= 2048


CASES = [
    ("adv2d_q1_1024x1024", lambda: random_scalar_workload(2, 1, (1024, 1024))),
    ("euler2d_q2_512x256", lambda: random_euler_workload(2, 2, (512, 256))),
    ("euler2d_q3_384x256", lambda: random_euler_workload(2, 3, (384, 256))),
]


@pytest.mark.parametrize("label,make", CASES, ids=[c[0] for c in CASES])
def test_wide_strided_runs_stage_parity(label, make):
    # the vector line kernels (these meshes take the matrix-core tiles by
    # default), then the matrix-core tiles against the same oracle stage
    wl = make()
    assert takes_wide_runs(wl)
    ref = oracle_stage(wl)
    compare_stage(wl, dict(line_kernels=0), label=label + "-vector", tol=TOL, ref=ref)
    compare_stage(wl, dict(line_kernels=1), label=label + "-matrix", tol=TOL, ref=ref)
