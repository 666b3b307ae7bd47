"""Shared set-up of matching oracle / HIP problems for the parity tests."""
import sys

import numpy as np

from oracle import Mesh, Oracle, Params, Problem
from paper_2509_04673_amd import workloads as W


def rel_linf(a, b, floor=0.0):
    """max |a - b| / max(max |b|, floor) (per whole array); floor is the
    natural size of the quantity where the reference itself may vanish."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    scale = max(float(np.max(np.abs(b))), floor)
    return float(np.max(np.abs(a - b)) / (scale if scale > 0 else 1.0))


def rel_l1(a, b, mass):
    """max over components of sum_i m_i |a - b| / sum_i m_i |b| (lumped
    nodal masses m_i)."""
    a = np.asarray(a, dtype=np.float64).reshape(-1, mass.size)
    b = np.asarray(b, dtype=np.float64).reshape(-1, mass.size)
    num = np.sum(mass * np.abs(a - b), axis=1)
    den = np.sum(mass * np.abs(b), axis=1)
    return float(np.max(num / np.where(den > 0, den, 1.0)))


def lumped_mass(orc):
    """m_i = |E_i| |K| / (p+1)^d on the oracle's mesh."""
    mesh = orc.mesh
    return mesh.multiplicity() * mesh.h ** mesh.d / mesh.nloc


def oracle_for(wl, modes=None, bounds=None):
    mesh = Mesh(wl.d, wl.p, wl.n, wl.lo, wl.hi)
    prm = Params(w_lin=wl.w_lin, q=wl.q)
    for k, v in (modes or {}).items():
        setattr(prm, k, v)
    if bounds is None:
        bounds = (float(wl.u0.min()), float(wl.u0.max()))
    prob = Problem(mesh, wl.kind, wl.velocity, wl.gamma_gas, params=prm,
                   u_min=bounds[0], u_max=bounds[1])
    return Oracle(prob)


MODE_CODES = {"weno": 0, "limit": 0, "zero": 1, "one": 2}


def gpu_for(wl, modes=None, precision="fp64"):
    from paper_2509_04673_amd.cem import Solver
    kw = {}
    for k, v in (modes or {}).items():
        kw[k] = v if k == "flux_mode" else MODE_CODES[v]
    s = Solver.from_workload(wl, precision=precision, **kw)
    s.upload(wl.u0)
    if wl.kind != "euler":
        s.set_bounds()
    return s


def announce(msg):
    print(msg, flush=True)
    sys.stdout.flush()


STAGE_TAPS = ["g", "gamma", "nu", "dt_e", "ue", "ubarL", "fA", "r", "udot", "ubar", "beta"]


def compare_stage(wl, modes=None, label="", tol=1e-12, floors=None):
    """One forward-Euler stage on the GPU and in the oracle from the same
    state: relative L-infinity error of every intermediate and of the stage
    result (which includes the bounds policy).  floors: per-tap lower bounds
    of the error scale (see rel_linf)."""
    orc = oracle_for(wl, modes)
    dt = wl.dt if wl.dt > 0 else 0.5 * orc.max_dt(wl.u0)
    announce(f"[parity] stage {label} d={wl.d} p={wl.p} n={wl.n} kind={wl.kind} modes={modes}")
    ufe, taps = orc.fe_stage(wl.u0, dt)
    ufe = orc.clamp(ufe)[0]
    s = gpu_for(wl, modes)
    s.stage(0, dt=dt)
    got = s.download()
    errs = {}
    for name in STAGE_TAPS:
        errs[name] = rel_linf(s.tap(name).reshape(np.shape(taps[name])), taps[name],
                              (floors or {}).get(name, 0.0))
    errs["u_fe"] = rel_linf(got, ufe)
    s.close()
    announce(f"[parity] {label}: " + ", ".join(f"{k}={v:.1e}" for k, v in errs.items()))
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, (label, errs)
    return errs, taps


def _perturbed(u):
    rng = np.random.default_rng(12345)
    return u * (1.0 + rng.integers(-1, 2, u.shape) * 2.0 ** -52)


def run_both(wl, nsteps, dt=None, cfl=0.5, modes=None):
    """GPU and oracle runs plus the oracle's own sensitivity floor: the
    divergence after nsteps caused by perturbing the input by 1 ulp."""
    orc = oracle_for(wl, modes)
    announce(f"[parity] {nsteps} steps {wl.name} n={wl.n} modes={modes}")
    u_ref, st = orc.run(wl.u0.copy(), nsteps, dt=dt, cfl=cfl)
    u_pert, _ = orc.run(_perturbed(wl.u0), nsteps, dt=dt, cfl=cfl)
    floor = rel_linf(u_pert, u_ref)
    s = gpu_for(wl, modes)
    for _ in range(nsteps):
        s.step(dt=dt or 0.0, cfl=0.0 if dt else cfl)
    got = s.download()
    chk = s.check()
    s.close()
    err = rel_linf(got, u_ref)
    announce(f"[parity] {wl.name}: rel Linf GPU vs oracle {err:.3e}, oracle 1-ulp floor {floor:.3e}")
    return err, floor, st, chk


def run_tol(floor):
    """1e-12, unless the scheme itself amplifies a 1-ulp input change beyond
    it over the run; the HIP path differs from the oracle by a few ulps per
    stage, so it may sit within a small multiple of that floor."""
    return max(1e-12, 20.0 * floor)


def random_scalar_workload(d, p, n, kind="advection", seed=0):
    """Rough data: smooth background, plateaus and noise (all sensor regimes)."""
    rng = np.random.default_rng(seed)
    lo = (0.0,) * d
    hi = tuple(float(nk) / max(n) for nk in n)
    x = W.node_coords(d, p, n, lo, hi)
    u = np.sin(2 * np.pi * x[:, 0] / hi[0]) + 0.3 * rng.standard_normal(x.shape[0]) * (x[:, 0] > 0.5 * hi[0])
    u = np.where(np.abs(x[:, -1] - 0.3 * hi[-1]) < 0.1 * hi[-1], 1.5, u)
    if kind == "kpp":
        u = 0.25 * np.pi + (3.25 * np.pi) * (u > 0.5)
    vel = (1.0, -0.5, 0.25)
    return W.Workload("rand", d, p, tuple(n), lo, hi, kind, u[None, :], velocity=vel,
                      w_lin=0.2 if (kind == "kpp") else 1e-3)


def random_euler_workload(d, p, n, seed=0):
    rng = np.random.default_rng(seed)
    lo = (0.0,) * d
    hi = tuple(float(nk) / max(n) for nk in n)
    x = W.node_coords(d, p, n, lo, hi)
    N = x.shape[0]
    blob = np.exp(-30 * np.sum((x - 0.4 * np.array(hi)) ** 2, axis=1))
    rho = 1.0 + 0.5 * blob + 0.2 * (x[:, 0] > 0.6 * hi[0])
    vel = [0.3 * np.sin(2 * np.pi * x[:, k] / hi[k]) for k in range(d)]
    pr = 1.0 + 5.0 * blob + 0.05 * rng.random(N)
    u = W._conserved(rho, vel, pr, 1.4)
    return W.Workload("rand_euler", d, p, tuple(n), lo, hi, "euler", u, w_lin=1e-3)
