"""Shared set-up of matching oracle / HIP problems for the parity tests."""
import os
import sys

import numpy as np

from oracle import Mesh, Oracle, Params, Problem
from paper_2509_04673_amd import workloads as W


def quantity_groups(m):
    """Components that form one physical quantity: Euler (m = d + 2) has
    density, the momentum vector and energy; a scalar problem one."""
    if m < 3:
        return [[c] for c in range(m)]
    return [[0], list(range(1, m - 1)), [m - 1]]


def rel_linf(a, b, floor=0.0):
    """Relative L-infinity error per physical quantity.

    Arrays shaped (..., m, X) (components on the second-to-last axis, nodes
    or elements last; leading axes such as the direction of g or f^A) are
    split into the quantities of quantity_groups: density, the momentum
    vector and energy for Euler.  Each quantity's error max |a - b| is
    divided by its own size max |b| over all its entries (a vector quantity,
    such as momentum or the gradient of one component, is measured against
    its magnitude, which no rotation changes), or by floor where that is
    larger (the natural size of a quantity whose reference may vanish); a
    quantity whose reference is exactly zero is measured against the largest
    one.  The result is the largest of these.  1-D arrays (per-element
    scalars) are one quantity."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    if a.size == 0:
        return 0.0
    if a.ndim < 2:
        a3, b3 = a.reshape(1, 1, -1), b.reshape(1, 1, -1)
    else:
        m = a.shape[-2]
        a3, b3 = a.reshape(-1, m, a.shape[-1]), b.reshape(-1, m, b.shape[-1])
    whole = max(float(np.max(np.abs(b3))), floor)
    worst = 0.0
    for grp in quantity_groups(a3.shape[1]):
        x, y = a3[:, grp, :], b3[:, grp, :]
        scale = max(float(np.max(np.abs(y))), floor)
        if scale == 0.0:
            scale = whole if whole > 0 else 1.0
        worst = max(worst, float(np.max(np.abs(x - y))) / scale)
    return worst


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


# switches of the HIP path alone (kernel choices with the same results)
GPU_ONLY = ("line_kernels",)


def state_bounds(wl):
    """Global bounds of a scalar workload as cem_set_bounds takes them from
    the state: the range of the coefficients and of any prescribed boundary
    state of a non-periodic line."""
    lo, hi = float(wl.u0.min()), float(wl.u0.max())
    for kind, state in (getattr(wl, "bc", None) or ()):
        if kind == "state":
            lo, hi = min(lo, float(state[0])), max(hi, float(state[0]))
    return lo, hi


def oracle_for(wl, modes=None, bounds=None):
    bc = getattr(wl, "bc", None)
    mesh = Mesh(wl.d, wl.p, wl.n, wl.lo, wl.hi, periodic=bc is None)
    prm = Params(w_lin=wl.w_lin, q=wl.q)
    for k, v in (modes or {}).items():
        if k not in GPU_ONLY:
            setattr(prm, k, v)
    if bounds is None:
        bounds = state_bounds(wl)
    prob = Problem(mesh, wl.kind, wl.velocity, wl.gamma_gas, params=prm,
                   u_min=bounds[0], u_max=bounds[1], bc=bc)
    return Oracle(prob)


MODE_CODES = {"weno": 0, "limit": 0, "zero": 1, "one": 2}


def gpu_for(wl, modes=None, precision="fp64"):
    from paper_2509_04673_amd.cem import Solver
    kw = {}
    for k, v in (modes or {}).items():
        if k not in GPU_ONLY:
            kw[k] = v if k in ("flux_mode", "bounds", "contrib") else MODE_CODES[v]
    s = Solver.from_workload(wl, precision=precision, **kw)
    if "line_kernels" in (modes or {}):
        s.set_line_kernels(modes["line_kernels"])
    s.upload(wl.u0)
    if wl.kind != "euler":
        s.set_bounds()
    return s


def line_plan(wl, axis, precision="fp64"):
    """(run length factor re, runs per thread ky) that the strided line
    passes take along axis 1 or 2 of a single problem, restated from the
    launch rule: runs of 2P where the line holds 2P + 2W nodes and 2048
    tiles of 32 lines x 8P remain; then the longest tile (ky = 4, 2) that
    keeps 2048 tiles and fits 40 KB of LDS."""
    p, m = wl.p, wl.u0.shape[0]
    W = ({1: 30, 2: 44, 3: 57} if precision == "fp64" else {1: 18, 2: 26, 3: 32})[p]
    vb = 8 if precision == "fp64" else 4
    S = -(-(2 * W + 1) // (4 * p)) * (4 * p)
    L = [p * k for k in wl.n]
    ntrans = m * int(np.prod(L)) // L[axis]

    def blocks(R, ky):
        return -(-ntrans // 32) * -(-L[axis] // (8 * R * ky))

    re = 2 if (L[axis] >= 2 * p + 2 * W and blocks(2 * p, 1) >= 2048) else 1
    R = p * re
    for ky in (4, 2):
        if blocks(R, ky) >= 2048 and (8 * R * ky + S) * 32 * vb <= 40960:
            return re, ky
    return re, 1


def announce(msg):
    """Print a progress / measurement line (and append it to the file named
    by CEM_PARITY_LOG, when set, so that a run keeps the measured errors of
    passing tests too)."""
    print(msg, flush=True)
    sys.stdout.flush()
    path = os.environ.get("CEM_PARITY_LOG")
    if path:
        with open(path, "a") as fh:
            fh.write(msg + "\n")


STAGE_TAPS = ["g", "gamma", "nu", "dt_e", "ue", "ubarL", "fA", "r", "udot", "ubar", "beta"]


def oracle_stage(wl, modes=None):
    """The oracle's stage on the workload: (oracle, dt, clamped stage result,
    intermediates); dt is the workload's, else half the largest admissible."""
    orc = oracle_for(wl, modes)
    dt = wl.dt if wl.dt > 0 else 0.5 * orc.max_dt(wl.u0)
    ufe, taps = orc.fe_stage(wl.u0, dt)
    return orc, dt, orc.clamp(ufe)[0], taps


def mass_condition(orc):
    """2-norm condition number of the consistent mass matrix M_C of the
    oracle's mesh: the product over axes of those of the assembled periodic
    1D mass matrices (M_C is their Kronecker product)."""
    p, h = orc.mesh.p, orc.mesh.h
    G = orc.el.t1["mass"]
    kappa = 1.0
    for k in range(orc.mesh.d):
        L = orc.mesh.L[k]
        M = np.zeros((L, L))
        for e in range(orc.mesh.n[k]):
            idx = [(p * e + a) % L for a in range(p + 1)]
            M[np.ix_(idx, idx)] += h * G
        kappa *= np.linalg.cond(M)
    return float(kappa)


def compare_stage(wl, modes=None, label="", tol=1e-12, floors=None, ref=None):
    """One forward-Euler stage on the GPU and in the oracle from the same
    state: relative L-infinity error of every intermediate and of the stage
    result (which includes the bounds policy), per physical quantity.
    floors: per-tap lower bounds of the error scale (see rel_linf), or
    "whole" for a tap measured against its largest quantity; ref: a
    precomputed oracle_stage.

    udot = M_C^{-1} r is defined by float64 arithmetic only to about
    kappa(M_C) eps of its size (the perturbation bound of a linear solve;
    kappa ~ 14^d for p = 2, ~ 51^d for p = 3), whichever solver computes it:
    that tap is held to max(tol, 4 kappa eps).  beta is compared on the
    elements where float64 fixes it to the tolerance: contributions above
    1e-12 of the largest and a rounding sensitivity 4 eps |u| m / |f| below
    the tolerance (elsewhere beta is arbitrary and inert)."""
    announce(f"[parity] stage {label} d={wl.d} p={wl.p} n={wl.n} kind={wl.kind} modes={modes}")
    orc, dt, ufe, taps = ref if ref is not None else oracle_stage(wl, modes)
    tols = {name: tol for name in STAGE_TAPS + ["u_fe"]}
    tols["udot"] = max(tol, 4.0 * mass_condition(orc) * np.finfo(float).eps)
    floors = dict(floors or {})
    for name, f in list(floors.items()):
        if isinstance(f, str) and f == "whole":
            ref_arr = ufe if name == "u_fe" else taps[name]
            floors[name] = float(np.max(np.abs(ref_arr)))
    s = gpu_for(wl, modes)
    s.stage(0, dt=dt)
    got = s.download()
    errs = {}
    for name in STAGE_TAPS:
        # with the Q1 contributions the udot tap holds the low-order derivative
        ref_name = "udot_lo" if (name == "udot" and (modes or {}).get("contrib") == "q1") else name
        got_t = s.tap(name).reshape(np.shape(taps[ref_name]))
        ref_t = taps[ref_name]
        if name == "beta":
            # beta_e is a ratio of the element's bound gaps to its
            # contributions (eq. 55, Appendix A): the gap subtracts two
            # rounded values, so a rounding change of ubar^e moves beta by up
            # to about 4 eps |u| m_i / |f_i^e|.  Where that exceeds
            # the tolerance (contributions that are rounding noise, or an
            # average at its bound to the last ulp) float64 does not fix
            # beta, and beta f_i^e / m_i changes the state only at rounding
            # level (u_fe is compared everywhere)
            fmax = np.max(np.abs(taps["fe"]), axis=(0, 2))
            mloc = orc.mesh.h ** orc.mesh.d / orc.mesh.nloc
            size = np.max(np.abs(taps["ubar"]), axis=0)
            if wl.kind != "euler":
                size = np.maximum(size, np.maximum(np.abs(taps["b_lo"]), np.abs(taps["b_hi"])))
            with np.errstate(divide="ignore"):
                sens = 4.0 * np.finfo(float).eps * size * mloc / fmax
            live = (fmax > 1e-12 * max(float(np.max(fmax)), 1e-300)) & (sens <= tols["beta"])
            got_t, ref_t = got_t[live], ref_t[live]
        errs[name] = rel_linf(got_t, ref_t, floors.get(name, 0.0))
    errs["u_fe"] = rel_linf(got, ufe, floors.get("u_fe", 0.0))
    if (modes or {}).get("bounds") == "local":
        tols["bounds"] = tol
        errs["bounds"] = rel_linf(s.tap("bounds").reshape(2, -1), np.stack([taps["b_lo"], taps["b_hi"]]))
    s.close()
    announce(f"[parity] {label}: " + ", ".join(f"{k}={v:.1e}" for k, v in errs.items())
             + f" (udot held to {tols['udot']:.1e})")
    bad = {k: v for k, v in errs.items() if not v <= tols[k]}
    assert not bad, (label, errs)
    return errs, taps


def _perturbed(u, seed=12345):
    rng = np.random.default_rng(seed)
    return u * (1.0 + rng.integers(-1, 2, u.shape) * 2.0 ** -52)


def run_both(wl, nsteps, dt=None, cfl=0.5, modes=None):
    """GPU and oracle runs plus the oracle's own sensitivity floor: the
    largest divergence after nsteps caused by perturbing the input by 1 ulp
    (two independent perturbations: the GPU's rounding differs at every
    stage, not in one input, and one sample can understate the spread)."""
    orc = oracle_for(wl, modes)
    announce(f"[parity] {nsteps} steps {wl.name} n={wl.n} modes={modes}")
    u_ref, st = orc.run(wl.u0.copy(), nsteps, dt=dt, cfl=cfl)
    floor = 0.0
    for seed in (12345, 54321):
        u_pert, _ = orc.run(_perturbed(wl.u0, seed), nsteps, dt=dt, cfl=cfl)
        floor = max(floor, rel_linf(u_pert, u_ref))
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
    it over the run (limiter and sensor switching): then the oracle's own
    response to that change, the spread any float64 evaluation order has."""
    return max(1e-12, floor)


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
