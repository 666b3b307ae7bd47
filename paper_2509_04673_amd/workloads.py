"""Seeded synthetic workloads: mesh, physics, parameters and initial data.

This module holds no arithmetic of the method.  It draws the seeded
parameters of each workload with splitmix64 and evaluates the initial data
u_0 at the Bernstein nodal points, u_j(0) = u_0(x_j) (nodal initialisation
of the numerical study, [KHV §5]).  Both the HIP path and the oracle consume
the arrays it returns.

Workloads (shapes of the paper's test problems):
  adv1d      1D linear advection, P2, periodic [0,1]: sin(2 pi x) plus a
             square pulse on [0.3, 0.5] of seeded amplitude in [0.5, 1]
  kpp2d      2D KPP flux (sin u, cos u) on [-2,2]x[-2.5,1.5], Q2:
             u = 7 pi / 2 in a radius-1 disc (seeded centre +-0.05),
             pi / 4 outside
  euler2d    2D Euler, gamma = 1.4, unit square, Q3: four quadrants with
             seeded rho, p in [0.1, 2] and velocities in [-1, 1]
  euler3d    3D Euler, unit cube, Q2: rho = 1, v = 0, p = 1e-2, p = 10
             inside a radius-0.1 ball at a seeded centre

Non-periodic 1D lines (the paper's 1D boundary tests, Sec. 5.1-5.2):
  inflow1d   linear advection on [0,1], v = 1: the step-and-bump profile of
             the 1D advection test, inflow state 0 at x = 0, outflow at 1
  sod1d      modified Sod shock tube on [0,1]: (1, 0.75, 1) left of the
             interface (0.25 + seeded shift below h/4), (0.125, 0, 0.1)
             right of it; the initial states as boundary data at both ends
  blast1d    Woodward-Colella blast wave on [0,1]: rho = 1, v = 0, p = 1000
             / 0.01 / 100 split at 0.1 and 0.9, reflecting walls
  shuosher1d Shu-Osher on [-5,5]: (3.857143, 2.629369, 10.33333) left of
             x = -4, (1 + 0.2 sin(5x), 0, 1) right of it, u_hat = u at both
             ends
  nonconvex1d the nonconvex flux of Sec. 5.1.2 on [0,1]: u_0 = 1 from
             x = 1/4 (+ a seeded shift below h/4), inflow state 0 at x = 0,
             outflow at x = 1
  line_batch many Sod, blast and Shu-Osher lines of 64..512 cells (the
             batched form)
"""
from dataclasses import dataclass, field
import math

import numpy as np

_MASK = (1 << 64) - 1


class SplitMix64:
    """splitmix64 (Steele, Lea & Flood 2014); uniforms (x >> 11) * 2^-53."""

    def __init__(self, seed):
        self.state = int(seed) & _MASK

    def next_u64(self):
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def uniform(self):
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)


@dataclass
class Workload:
    name: str
    d: int
    p: int
    n: tuple
    lo: tuple
    hi: tuple
    kind: str                       # "advection" | "kpp" | "euler" | "nonconvex"
    u0: np.ndarray                  # (m, N) float64, component-major, x fastest
    velocity: tuple = (1.0, 0.0, 0.0)
    gamma_gas: float = 1.4
    w_lin: float = 1e-3
    q: float = 1.0
    dt: float = 0.0                 # > 0: fixed step; 0: adaptive
    cfl: float = 0.5
    nsteps: int = 1
    meta: dict = field(default_factory=dict)
    # None: periodic; else ((kind, state), (kind, state)) of a 1D line's ends
    bc: tuple = None

    @property
    def m(self):
        return self.u0.shape[0]

    @property
    def N(self):
        return self.u0.shape[1]

    @property
    def dofs(self):
        return self.u0.size


def node_coords(d, p, n, lo, hi, periodic=True):
    """(N, d) nodal points x_j = lo + h i / p on the periodic node lattice
    (or the p n + 1 points of a non-periodic line), x fastest (node index
    sum_k i_k prod_{j<k} L_j)."""
    L = [p * nk + (0 if periodic else 1) for nk in n]
    h = [(hi[k] - lo[k]) / n[k] for k in range(d)]
    axes = [lo[k] + h[k] * np.arange(L[k]) / p for k in range(d)]
    grids = np.meshgrid(*reversed(axes), indexing="ij")    # slowest first
    return np.stack([g.ravel() for g in reversed(grids)], axis=1)


def _conserved(rho, vel, pres, gamma):
    """(rho, rho v, rho E) from primitive variables of an ideal gas
    (equation of state of [KHV §5.2])."""
    d = len(vel)
    kin = 0.5 * rho * sum(v * v for v in vel)
    return np.stack([rho] + [rho * v for v in vel] + [pres / (gamma - 1.0) + kin])


def adv1d(seed=0, n=64, p=2):
    rng = SplitMix64(seed)
    amp = 0.5 + 0.5 * rng.uniform()
    x = node_coords(1, p, (n,), (0.0,), (1.0,))[:, 0]
    u = np.sin(2.0 * math.pi * x) + amp * ((x >= 0.3) & (x <= 0.5))
    return Workload("adv1d", 1, p, (n,), (0.0,), (1.0,), "advection", u[None, :],
                    velocity=(1.0, 0.0, 0.0), w_lin=1e-3, dt=0.2 * (1.0 / n) / 2.0,
                    cfl=0.2, nsteps=200, meta=dict(amplitude=amp, seed=seed))


def kpp2d(seed=0, n=256, p=2):
    rng = SplitMix64(seed)
    cx = -0.05 + 0.1 * rng.uniform()
    cy = -0.05 + 0.1 * rng.uniform()
    lo, hi = (-2.0, -2.5), (2.0, 1.5)
    xy = node_coords(2, p, (n, n), lo, hi)
    r2 = (xy[:, 0] - cx) ** 2 + (xy[:, 1] - cy) ** 2
    u = np.where(r2 <= 1.0, 3.5 * math.pi, 0.25 * math.pi)
    return Workload("kpp2d", 2, p, (n, n), lo, hi, "kpp", u[None, :], w_lin=0.2,
                    dt=5e-4, nsteps=2000, meta=dict(centre=(cx, cy), seed=seed))


def _quadrant_states(rng):
    """(rho, vx, vy, p) per quadrant, drawn in the order NE, NW, SW, SE."""
    out = []
    for _ in range(4):
        rho = 0.1 + 1.9 * rng.uniform()
        vx = -1.0 + 2.0 * rng.uniform()
        vy = -1.0 + 2.0 * rng.uniform()
        pr = 0.1 + 1.9 * rng.uniform()
        out.append((rho, vx, vy, pr))
    return out


def euler2d(seed=0, n=512, p=3, gamma=1.4):
    rng = SplitMix64(seed)
    st = _quadrant_states(rng)
    xy = node_coords(2, p, (n, n), (0.0, 0.0), (1.0, 1.0))
    east = xy[:, 0] >= 0.5
    north = xy[:, 1] >= 0.5
    q = np.where(north, np.where(east, 0, 1), np.where(east, 3, 2))
    prim = np.array(st)[q]                      # (N, 4)
    u = _conserved(prim[:, 0], [prim[:, 1], prim[:, 2]], prim[:, 3], gamma)
    return Workload("euler2d", 2, p, (n, n), (0.0, 0.0), (1.0, 1.0), "euler", u,
                    gamma_gas=gamma, w_lin=1e-3, dt=0.0, cfl=0.5, nsteps=100,
                    meta=dict(quadrants=st, seed=seed))


def euler3d(seed=0, n=128, p=2, gamma=1.4):
    rng = SplitMix64(seed)
    c = [0.2 + 0.6 * rng.uniform() for _ in range(3)]
    xyz = node_coords(3, p, (n, n, n), (0.0,) * 3, (1.0,) * 3)
    r2 = sum((xyz[:, k] - c[k]) ** 2 for k in range(3))
    pres = np.where(r2 <= 0.01, 10.0, 1e-2)
    rho = np.ones_like(pres)
    z = np.zeros_like(pres)
    u = _conserved(rho, [z, z, z], pres, gamma)
    return Workload("euler3d", 3, p, (n, n, n), (0.0,) * 3, (1.0,) * 3, "euler", u,
                    gamma_gas=gamma, w_lin=1e-3, dt=0.0, cfl=0.5, nsteps=500,
                    meta=dict(centre=c, seed=seed))


def euler_batch_sizes(seed=0, count=512):
    """Mesh sizes n_k = 32 + floor(225 U) of the batched Euler workload."""
    rng = SplitMix64(seed)
    return [32 + int(225 * rng.uniform()) for _ in range(count)]


def euler_batch_octiles(seed=0, count=512):
    """Indices of eight problems of the batched workload that span its size
    range: the smallest, the largest and the six octiles between them (by
    mesh size, first index among equal sizes)."""
    sizes = euler_batch_sizes(seed, count)
    order = sorted(range(count), key=lambda k: (sizes[k], k))
    return [order[round(q * (count - 1) / 7)] for q in range(8)]


def euler_batch(seed=0, count=512, p=2, gamma=1.4, sizes=None, only=None):
    """The batched Euler workload: count independent four-quadrant problems
    on the unit square, Q2, square n_k^2 meshes with n_k = 32 + floor(225 U)
    (drawn first), then each problem's quadrant states (NE, NW, SW, SE; rho,
    vx, vy, p per quadrant) from the same generator.  only: indices of the
    problems to build (the draws of all problems still happen in order)."""
    rng = SplitMix64(seed)
    if sizes is None:
        sizes = [32 + int(225 * rng.uniform()) for _ in range(count)]
    out = []
    for k, n in enumerate(sizes):
        st = _quadrant_states(rng)
        if only is not None and k not in only:
            continue
        xy = node_coords(2, p, (n, n), (0.0, 0.0), (1.0, 1.0))
        east = xy[:, 0] >= 0.5
        north = xy[:, 1] >= 0.5
        q = np.where(north, np.where(east, 0, 1), np.where(east, 3, 2))
        prim = np.array(st)[q]
        u = _conserved(prim[:, 0], [prim[:, 1], prim[:, 2]], prim[:, 3], gamma)
        out.append(Workload(f"euler_batch[{k}]", 2, p, (n, n), (0.0, 0.0), (1.0, 1.0), "euler", u,
                            gamma_gas=gamma, w_lin=1e-3, dt=0.0, cfl=0.5, nsteps=50,
                            meta=dict(quadrants=st, seed=seed, index=k)))
    return out


MAKERS = dict(adv1d=adv1d, kpp2d=kpp2d, euler2d=euler2d, euler3d=euler3d)


def make(name, seed=0, **kw):
    return MAKERS[name](seed=seed, **kw)


# ---------------------------------------------------------------------------
# non-periodic 1D lines
# ---------------------------------------------------------------------------
def _line_x(p, n, lo, hi):
    return node_coords(1, p, (n,), (lo,), (hi,), periodic=False)[:, 0]


def inflow1d(seed=0, n=128, p=1):
    rng = SplitMix64(seed)
    shift = 0.01 * (rng.uniform() - 0.5)
    x = _line_x(p, n, 0.0, 1.0) - shift
    bump = np.zeros_like(x)
    inside = (x > 0.5) & (x < 0.9)
    xi = x[inside]
    bump[inside] = np.exp(10.0 + 1.0 / (0.5 - xi) + 1.0 / (xi - 0.9))
    u = np.where((x >= 0.2) & (x <= 0.4), 1.0, bump)
    return Workload("inflow1d", 1, p, (n,), (0.0,), (1.0,), "advection", u[None, :],
                    velocity=(1.0, 0.0, 0.0), dt=0.0, cfl=0.5, nsteps=100,
                    meta=dict(shift=shift, seed=seed), bc=(("state", [0.0]), ("outflow", None)))


def _line_euler(name, p, n, lo, hi, prim, gamma, nsteps, bc_kind, meta):
    u = _conserved(prim[0], [prim[1]], prim[2], gamma)
    if bc_kind == "state":
        bc = (("state", u[:, 0].copy()), ("state", u[:, -1].copy()))
    else:
        bc = ((bc_kind, None), (bc_kind, None))
    return Workload(name, 1, p, (n,), (lo,), (hi,), "euler", u, gamma_gas=gamma, w_lin=1e-3,
                    dt=0.0, cfl=0.5, nsteps=nsteps, meta=meta, bc=bc)


def sod1d(seed=0, n=128, p=1, gamma=1.4):
    rng = SplitMix64(seed)
    h = 1.0 / n
    xs = 0.25 + 0.25 * h * (rng.uniform() - 0.5)
    x = _line_x(p, n, 0.0, 1.0)
    left = x < xs
    prim = (np.where(left, 1.0, 0.125), np.where(left, 0.75, 0.0), np.where(left, 1.0, 0.1))
    return _line_euler("sod1d", p, n, 0.0, 1.0, prim, gamma, 100, "state", dict(split=xs, seed=seed))


def blast1d(seed=0, n=1000, p=1, gamma=1.4):
    rng = SplitMix64(seed)
    h = 1.0 / n
    a = 0.1 + 0.25 * h * (rng.uniform() - 0.5)
    b = 0.9 + 0.25 * h * (rng.uniform() - 0.5)
    x = _line_x(p, n, 0.0, 1.0)
    pr = np.where(x < a, 1000.0, np.where(x > b, 100.0, 0.01))
    prim = (np.ones_like(x), np.zeros_like(x), pr)
    return _line_euler("blast1d", p, n, 0.0, 1.0, prim, gamma, 100, "wall", dict(splits=(a, b), seed=seed))


def shuosher1d(seed=0, n=500, p=1, gamma=1.4):
    rng = SplitMix64(seed)
    h = 10.0 / n
    xs = -4.0 + 0.25 * h * (rng.uniform() - 0.5)
    x = _line_x(p, n, -5.0, 5.0)
    left = x < xs
    prim = (np.where(left, 3.857143, 1.0 + 0.2 * np.sin(5.0 * x)), np.where(left, 2.629369, 0.0),
            np.where(left, 10.33333, 1.0))
    return _line_euler("shuosher1d", p, n, -5.0, 5.0, prim, gamma, 100, "outflow", dict(split=xs, seed=seed))


def nonconvex1d(seed=0, n=128, p=1):
    rng = SplitMix64(seed)
    h = 1.0 / n
    xs = 0.25 + 0.25 * h * (rng.uniform() - 0.5)
    x = _line_x(p, n, 0.0, 1.0)
    u = (x >= xs).astype(np.float64)
    return Workload("nonconvex1d", 1, p, (n,), (0.0,), (1.0,), "nonconvex", u[None, :], dt=0.0, cfl=0.5,
                    nsteps=100, meta=dict(split=xs, seed=seed), bc=(("state", [0.0]), ("outflow", None)))


MAKERS.update(inflow1d=inflow1d, sod1d=sod1d, blast1d=blast1d, shuosher1d=shuosher1d, nonconvex1d=nonconvex1d)


def line_batch(seed=0, count=4096, p=2):
    """Many independent Euler lines of the paper's 1D boundary tests for
    the batched form: problem k is the modified Sod tube, the blast wave or
    the Shu-Osher problem (k mod 3) on n_k = 64 + floor(449 U) cells drawn
    from splitmix64 (seed), its own data seeded with k."""
    rng = SplitMix64(seed)
    makers = (sod1d, blast1d, shuosher1d)
    out = []
    for k in range(count):
        n = 64 + int(449 * rng.uniform())
        w = makers[k % 3](seed=k, n=n, p=p)
        w.name = f"line_batch[{k}]:{w.name}"
        out.append(w)
    return out
