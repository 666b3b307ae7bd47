"""Writes the oracle's multi-step reference states used by
tests/test_gpu_runs.py (float64, SSP-RK3).

For each run: the seeded workload (paper_2509_04673_amd.workloads, inputs
only) advanced by the oracle for the stated number of steps, sampled at every
STRIDE-th node (all components), together with the oracle's own 1-ulp
floor: the same run from the input perturbed by one ulp at random nodes
(seeded), measured on the same samples with the per-quantity relative
L-infinity and L1 errors of the tests; and the float floor: the relative L1
response to a float-sized input perturbation (the rounding the mixed form
adds at every stage).  Only the oracle computes; nothing here calls
the HIP library.

Usage: python tests/golden/make_runs.py [name ...]   (default: all runs)
Each run takes minutes to an hour of one core (the 3D run is the longest).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

from oracle import Mesh, Oracle, Params, Problem          # noqa: E402
from paper_2509_04673_amd import workloads as W           # noqa: E402

# name: (workload maker, steps, node stride of the samples)
RUNS = {
    "kpp2d_256x256_q2_100steps": (lambda: W.kpp2d(seed=0, n=256), 100, 7),
    "euler2d_64x64_q3_20steps": (lambda: W.euler2d(seed=0, n=64), 20, 3),
    "euler3d_32x32x32_q2_50steps": (lambda: W.euler3d(seed=0, n=32), 50, 29),
}


def oracle_for(wl):
    mesh = Mesh(wl.d, wl.p, wl.n, wl.lo, wl.hi)
    prm = Params(w_lin=wl.w_lin, q=wl.q)
    return Oracle(Problem(mesh, wl.kind, wl.velocity, wl.gamma_gas, params=prm,
                          u_min=float(wl.u0.min()), u_max=float(wl.u0.max())))


def perturbed(u):
    rng = np.random.default_rng(12345)
    return u * (1.0 + rng.integers(-1, 2, u.shape) * 2.0 ** -52)


def float_perturbed(u):
    """The input moved by float-sized relative amounts (uniform in
    +-2^-24): the size of what the mixed form rounds at every stage."""
    rng = np.random.default_rng(7)
    return u * (1.0 + rng.uniform(-1.0, 1.0, u.shape) * 2.0 ** -24)


def rel_linf_groups(a, b):
    """Per-quantity relative L-infinity error (density, momentum, energy for
    Euler; the one component of a scalar problem), the largest."""
    m = a.shape[0]
    groups = [[c] for c in range(m)] if m < 3 else [[0], list(range(1, m - 1)), [m - 1]]
    return max(float(np.max(np.abs(a[g] - b[g])) / np.max(np.abs(b[g]))) for g in groups)


def sample_mass(mesh, sel):
    """Lumped masses m_i = |E_i| |K| / (p+1)^d of the sampled nodes."""
    return mesh.multiplicity()[sel] * mesh.h ** mesh.d / mesh.nloc


def rel_l1_groups(a, b, mass):
    """Per-quantity relative L1 error sum m_i |a - b| / sum m_i |b| (over
    all components of the quantity), the largest."""
    m = a.shape[0]
    groups = [[c] for c in range(m)] if m < 3 else [[0], list(range(1, m - 1)), [m - 1]]
    return max(float(np.sum(mass * np.abs(a[g] - b[g])) / np.sum(mass * np.abs(b[g]))) for g in groups)


def make(name):
    mk, steps, stride = RUNS[name]
    wl = mk()
    orc = oracle_for(wl)
    dt = wl.dt if wl.dt > 0 else None
    t0 = time.time()
    ref, st = orc.run(wl.u0.copy(), steps, dt=dt, cfl=wl.cfl)
    pert, _ = orc.run(perturbed(wl.u0), steps, dt=dt, cfl=wl.cfl)
    sel = np.arange(0, wl.N, stride)
    floor = rel_linf_groups(pert[:, sel], ref[:, sel])
    mass = sample_mass(orc.mesh, sel)
    floor_l1 = rel_l1_groups(pert[:, sel], ref[:, sel], mass)
    fpert, _ = orc.run(float_perturbed(wl.u0), steps, dt=dt, cfl=wl.cfl)
    floor_f32_l1 = rel_l1_groups(fpert[:, sel], ref[:, sel], mass)
    out = os.path.join(HERE, f"run_{name}.npz")
    np.savez_compressed(out, samples=ref[:, sel], stride=stride, steps=steps, floor=floor,
                        floor_l1=floor_l1, floor_f32_l1=floor_f32_l1, violations=st["violations"],
                        clamped=st["clamped"], dt=-1.0 if dt is None else dt, cfl=wl.cfl)
    print(f"{name}: {steps} steps, {sel.size} sampled nodes, 1-ulp floor rel Linf {floor:.3e}, "
          f"rel L1 {floor_l1:.3e}; float-input floor rel L1 {floor_f32_l1:.3e}; violations "
          f"{st['violations']}, {time.time() - t0:.0f} s -> {out}", flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(RUNS)):
        make(n)
