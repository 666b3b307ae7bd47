"""Non-periodic 1D lines on the GPU against the oracle: the boundary term
b_i of eq. (bidef), the boundary facet fluxes f^partial and f^L of Sec. 4,
g_i^e of eq. (aecb), one-sided flux limiting at boundary facets (eq. 53,
e' > E_h), absent WENO candidates and the line operators of the bounded
mass matrix.

Tolerances: one stage, relative L-infinity 1e-12 per intermediate and for
the stage result (udot to 4 kappa(M) eps, as on periodic meshes); runs
within the oracle's own 1-ulp sensitivity floor.  Cases span short lines
(every line-operator row exact) and long ones (exact end blocks, infinite-
line rows inside), every boundary kind, both physics and p = 1..3."""
import numpy as np
import pytest

from paper_2509_04673_amd import workloads as W
from parity_util import (announce, compare_stage, gpu_for, lumped_mass, oracle_for, random_euler_workload,
                         random_scalar_workload, rel_linf, run_both, run_tol)

pytestmark = pytest.mark.gpu

TOL = 1e-12


def line_workload(kind, p, n, bc, seed=0, velocity=1.0):
    """Rough data on [0, 1] (plateaus, noise, a smooth part) with the given
    boundary kinds; prescribed states are drawn near the interior data."""
    rng = np.random.default_rng(seed)
    x = W.node_coords(1, p, (n,), (0.0,), (1.0,), periodic=False)[:, 0]
    if kind != "euler":
        u = np.sin(2 * np.pi * x) + 0.3 * rng.standard_normal(x.size) * (x > 0.5)
        u = np.where(np.abs(x - 0.3) < 0.1, 1.5, u)
        u = u[None]
        st = lambda: [float(rng.uniform(-1.0, 1.8))]
    else:
        rho = 1.0 + 0.5 * np.exp(-30 * (x - 0.4) ** 2) + 0.4 * (x > 0.7)
        v = 0.4 * np.sin(3 * np.pi * x) + 0.05 * rng.standard_normal(x.size)
        pr = 1.0 + 3.0 * (x < 0.2) + 0.05 * rng.random(x.size)
        u = W._conserved(rho, [v], pr, 1.4)
        st = lambda: list(W._conserved(np.array([rng.uniform(0.5, 2.0)]), [np.array([rng.uniform(-0.5, 0.5)])],
                                       np.array([rng.uniform(0.5, 3.0)]), 1.4)[:, 0])
    bcs = tuple((k, st() if k == "state" else None) for k in bc)
    return W.Workload(f"line_{kind}", 1, p, (n,), (0.0,), (1.0,), kind, u, velocity=(velocity, 0.0, 0.0),
                      w_lin=1e-3, bc=bcs)


CASES = [
    ("adv_p1_in_out", lambda: line_workload("advection", 1, 41, ("state", "outflow"))),
    ("adv_p2_out_in", lambda: line_workload("advection", 2, 23, ("outflow", "state"), velocity=-0.7)),
    ("adv_p3_state_state", lambda: line_workload("advection", 3, 17, ("state", "state"), seed=2)),
    ("adv_p1_long", lambda: line_workload("advection", 1, 400, ("state", "outflow"), seed=3)),
    ("adv_p2_long", lambda: line_workload("advection", 2, 200, ("state", "outflow"), seed=4)),
    ("adv_p3_long", lambda: line_workload("advection", 3, 150, ("outflow", "state"), seed=5, velocity=-1.0)),
    ("eul_p1_state_wall", lambda: line_workload("euler", 1, 40, ("state", "wall"))),
    ("eul_p2_wall_out", lambda: line_workload("euler", 2, 24, ("wall", "outflow"), seed=6)),
    ("eul_p3_out_state", lambda: line_workload("euler", 3, 15, ("outflow", "state"), seed=7)),
    ("eul_p2_long", lambda: line_workload("euler", 2, 300, ("state", "wall"), seed=8)),
    ("eul_p2_two_cells", lambda: line_workload("euler", 2, 2, ("wall", "wall"), seed=9)),
    ("sod_p1", lambda: W.sod1d(seed=1, n=64, p=1)),
    ("sod_p2", lambda: W.sod1d(seed=1, n=32, p=2)),
    ("blast_p1", lambda: W.blast1d(seed=1, n=100, p=1)),
    ("blast_p2", lambda: W.blast1d(seed=1, n=50, p=2)),
    ("shuosher_p2", lambda: W.shuosher1d(seed=1, n=60, p=2)),
    ("inflow_p3", lambda: W.inflow1d(seed=1, n=30, p=3)),
    ("ncv_p1", lambda: W.nonconvex1d(seed=1, n=64, p=1)),
    ("ncv_p2_long", lambda: W.nonconvex1d(seed=1, n=200, p=2)),
    ("ncv_p3_rough", lambda: line_workload("nonconvex", 3, 20, ("state", "outflow"), seed=12)),
    # either side of the shortest line that takes the banded layout (end
    # blocks + infinite rows): 62 / 46 / 40 cells for p = 1 / 2 / 3
    ("adv_p1_62_first_banded", lambda: line_workload("advection", 1, 62, ("outflow", "state"), seed=14,
                                                      velocity=-1.0)),
    ("eul_p2_46_first_banded", lambda: line_workload("euler", 2, 46, ("state", "wall"), seed=13)),
    ("eul_p2_45_last_dense", lambda: line_workload("euler", 2, 45, ("wall", "state"), seed=15)),
    ("ncv_p3_40_first_banded", lambda: line_workload("nonconvex", 3, 40, ("state", "outflow"), seed=16)),
]

MODES = [
    ("method", {}),
    ("target", dict(alpha_mode="one", beta_mode="one")),
    ("low_order", dict(gamma_mode="zero", alpha_mode="zero", beta_mode="zero")),
    ("shrink", dict(flux_mode="shrink")),
]


@pytest.mark.parametrize("mlabel,modes", MODES, ids=[m[0] for m in MODES])
@pytest.mark.parametrize("label,make", CASES, ids=[c[0] for c in CASES])
def test_line_stage_parity(label, make, mlabel, modes):
    wl = make()
    floors = None
    if label.startswith("blast"):
        # the blast wave starts with constant density and zero momentum: g,
        # r and udot of those components are rounding noise on both sides
        # (row sums of the line operators), measured against the largest
        # component (energy)
        floors = {"g": "whole", "r": "whole", "udot": "whole"}
    compare_stage(wl, modes, f"{label}-{mlabel}", TOL, floors=floors)


@pytest.mark.parametrize("label,make", [c for c in CASES if c[0].startswith(("adv", "inflow", "ncv"))],
                         ids=[c[0] for c in CASES if c[0].startswith(("adv", "inflow", "ncv"))])
def test_line_stage_parity_local_bounds(label, make):
    wl = make()
    errs, taps = compare_stage(wl, dict(bounds="local"), f"{label}-local", TOL)
    # the inflow element's bounds reach its boundary data
    assert np.all(taps["ubar"][0] >= taps["b_lo"] - 1e-12) and np.all(taps["ubar"][0] <= taps["b_hi"] + 1e-12)


def test_line_stage_parity_at_two_thousand_nodes():
    compare_stage(line_workload("euler", 2, 1000, ("state", "outflow"), seed=11), {}, "eul_p2_1000", TOL)


RUNS = [
    ("sod_p2", lambda: W.sod1d(seed=2, n=64, p=2), 30),
    ("sod_p1", lambda: W.sod1d(seed=2, n=128, p=1), 30),
    ("blast_p1", lambda: W.blast1d(seed=2, n=200, p=1), 30),
    ("shuosher_p2", lambda: W.shuosher1d(seed=2, n=100, p=2), 30),
    ("inflow_p2", lambda: W.inflow1d(seed=2, n=64, p=2), 40),
    ("nonconvex_p1", lambda: W.nonconvex1d(seed=2, n=128, p=1), 40),
]


@pytest.mark.parametrize("label,make,nsteps", RUNS, ids=[r[0] for r in RUNS])
def test_line_run_parity(label, make, nsteps):
    wl = make()
    err, floor, st, chk = run_both(wl, nsteps, cfl=0.5)
    assert err <= run_tol(floor), (err, floor)
    assert chk["violations"] == 0 == st["violations"]
    assert not chk["cfl_violated"]


def test_walls_conserve_mass_and_energy_on_the_gpu():
    wl = W.blast1d(seed=3, n=400, p=2)
    s = gpu_for(wl)
    m = lumped_mass(oracle_for(wl))
    before = m @ wl.u0[0], m @ wl.u0[2]
    for _ in range(20):
        s.step(cfl=0.5)
    u = s.download()
    chk = s.check()
    s.close()
    dm = abs(m @ u[0] - before[0]) / before[0]
    de = abs(m @ u[2] - before[1]) / before[1]
    announce(f"[boundary] blast p2 400 cells, 20 steps: mass drift {dm:.1e}, energy drift {de:.1e}")
    assert dm <= 1e-13 and de <= 1e-13
    assert chk["violations"] == 0


def test_inflow_state_enters_the_bounds():
    from paper_2509_04673_amd.cem import CemError
    wl = W.inflow1d(seed=0, n=40, p=2)
    wl.bc = (("state", [1.7]), ("outflow", None))
    s = gpu_for(wl)                 # bounds from the state: [0, 1.7]
    with pytest.raises(CemError):
        s.set_bounds(0.0, 1.0)      # the inflow state would lie outside
    s.set_bounds(0.0, 1.7)
    for _ in range(30):
        s.step(cfl=0.5)
    u = s.download()
    chk = s.check()
    s.close()
    assert chk["violations"] == 0 and u.max() <= 1.7 + 1e-12 and u.min() >= -1e-12
    # the inflow state reaches the first node
    assert abs(u[0, 0] - 1.7) < 0.2


@pytest.mark.parametrize("p", [1, 2])
def test_nonconvex_riemann_problem_reaches_the_entropy_solution(p):
    # Sec. 5.1.2 with N_h = 129: the first 40 steps match the oracle within
    # its 1-ulp floor (over the whole run to t = 1 the limiter switching
    # amplifies rounding beyond what two perturbation samples bound); at
    # t = 1 the GPU's L1 distance to the exact entropy solution (shock from
    # 0 to sqrt(3/8), then the rarefaction) is that of the oracle's run
    from test_oracle_nonconvex import exact
    wl = W.nonconvex1d(seed=0, n=128 // p, p=p)
    orc = oracle_for(wl)
    dt0 = 0.5 * orc.max_dt(wl.u0)
    nsteps = int(np.ceil(1.0 / dt0))
    dt = 1.0 / nsteps
    err, floor, st, chk = run_both(wl, 40, dt=dt)
    assert err <= run_tol(floor), (err, floor)
    s = gpu_for(wl)
    for _ in range(nsteps):
        s.step(dt=dt)
    u = s.download()[0]
    chk = s.check()
    s.close()
    ref, _ = orc.run(wl.u0.copy(), nsteps, dt=dt)
    conn = np.arange(wl.n[0])[:, None] * p + np.arange(p + 1)[None, :]
    h = 1.0 / wl.n[0]
    tq, wq = np.polynomial.legendre.leggauss(8)
    ex = np.array([np.sum(wq * exact(e * h + h * (tq + 1) / 2, 1.0)) / 2 for e in range(wl.n[0])])
    l1 = h * np.sum(np.abs(u[conn].mean(axis=1) - ex))
    l1_ref = h * np.sum(np.abs(ref[0][conn].mean(axis=1) - ex))
    announce(f"[boundary] nonconvex Riemann problem p={p}, t = 1: L1 distance to the entropy solution "
             f"{l1:.3e} (oracle {l1_ref:.3e})")
    assert l1 < 1.5e-2 and abs(l1 - l1_ref) <= 0.02 * l1_ref
    assert chk["violations"] == 0


@pytest.mark.parametrize("p,n0,ratio", [(1, 100, 4.0), (2, 50, 1.8)])
def test_modified_sod_converges_to_the_exact_solution_on_the_gpu(p, n0, ratio):
    # Sec. 5.2.1 to t = 0.2: at n0 cells the GPU's L1 errors against the
    # exact entropy solution (every conserved variable, cell averages) are
    # the oracle's, within the oracle's own response to a 1-ulp change of
    # the data (the P1 run's limiter switching moves its state by 2-3% and
    # these errors by up to 4%; P2 by 1.6e-7); at 2, 4 and 8 n0
    # cells, where the oracle's runs would take minutes, they keep falling.
    # The oracle's own runs fall by 7.0 - 8.0 (P1) and 2.2 - 2.5 (P2, whose
    # rate drops from 1.4 to 1.2 per doubling at 400 cells) over the three
    # doublings: the thresholds ask for 4 and 1.8
    from exact_riemann import cell_averages
    from parity_util import _perturbed
    T = 0.2
    errs = []
    for n in (n0, 2 * n0, 4 * n0, 8 * n0):
        wl = W.sod1d(seed=3, n=n, p=p)
        orc = oracle_for(wl)
        k = int(np.ceil(T / (0.4 * orc.max_dt(wl.u0))))
        announce(f"[boundary] modified Sod p={p} n={n}: {k} steps to t = {T}")
        s = gpu_for(wl)
        for _ in range(k):
            s.step(dt=T / k)
        u = s.download()
        chk = s.check()
        s.close()
        assert chk["violations"] == 0 and not chk["cfl_violated"]
        conn = np.arange(n)[:, None] * p + np.arange(p + 1)[None, :]
        ex = cell_averages((1.0, 0.75, 1.0), (0.125, 0.0, 0.1), wl.meta["split"], T, np.linspace(0.0, 1.0, n + 1))
        l1 = lambda v: np.abs(v[:, conn].mean(axis=2) - ex).sum(axis=1) / n
        err = l1(u)
        if n == n0:
            ref_err = l1(orc.run(wl.u0.copy(), k, dt=T / k)[0])
            floor = 1e-9
            for seed in (12345, 54321):
                pert = l1(orc.run(_perturbed(wl.u0, seed), k, dt=T / k)[0])
                floor = max(floor, float(np.max(np.abs(pert - ref_err) / ref_err)))
            dev = np.abs(err - ref_err) / ref_err
            announce(f"[boundary]   L1 (rho, m, E) {err} (oracle {ref_err}); relative difference "
                     f"{dev.max():.2e}, oracle 1-ulp floor {floor:.2e}")
            # twice the larger of the two samples: the GPU's rounding differs
            # at every stage, and two draws bound that spread only roughly
            # (P2 measured 1.4e-7 against a floor of 1.6e-7)
            assert np.all(dev <= 2.0 * floor), (dev, floor)
        else:
            announce(f"[boundary]   L1 (rho, m, E) {err}")
        errs.append(err)
    assert all(np.all(b < a) for a, b in zip(errs, errs[1:]))
    assert np.all(errs[0] >= ratio * errs[-1]), errs[0] / errs[-1]


# -- batched form: many lines of uneven size and boundary kinds in one launch
# per kernel and stage
def _line_batch(wls):
    from paper_2509_04673_amd.cem import BatchSolver
    w0 = wls[0]
    b = BatchSolver([(w.d, w.p, w.n, w.lo, w.hi, w.bc) for w in wls], w0.kind, w0.velocity, w0.gamma_gas,
                    w_lin=w0.w_lin)
    b.upload([w.u0 for w in wls])
    if w0.kind != "euler":
        b.set_bounds()
    return b


BATCHES = [
    ("euler_p2", lambda: [W.sod1d(seed=1, n=40, p=2), W.blast1d(seed=1, n=100, p=2),
                          W.shuosher1d(seed=1, n=64, p=2), W.sod1d(seed=2, n=300, p=2),
                          line_workload("euler", 2, 24, ("state", "wall"), seed=13)]),
    ("euler_p1", lambda: [W.blast1d(seed=3, n=2, p=1), W.sod1d(seed=3, n=129, p=1), W.shuosher1d(seed=3, n=400, p=1)]),
    ("nonconvex_p3", lambda: [W.nonconvex1d(seed=4, n=n, p=3) for n in (5, 33, 120)]),
    # periodic lines through the same batched launches
    ("periodic_euler_p2", lambda: [random_euler_workload(1, 2, (n,), seed=n) for n in (3, 40, 700)]),
    ("periodic_adv_p3", lambda: [random_scalar_workload(1, 3, (n,), seed=n) for n in (4, 50, 300)]),
]


@pytest.mark.parametrize("label,make", BATCHES, ids=[b[0] for b in BATCHES])
def test_line_batch_matches_the_oracle(label, make):
    wls = make()
    b = _line_batch(wls)
    b.step(cfl=0.5, nsteps=2)
    got = b.download()
    chk = b.check()
    b.close()
    for k, (w, g, c) in enumerate(zip(wls, got, chk)):
        orc = oracle_for(w)
        ref, st = orc.run(w.u0.copy(), 2, cfl=0.5)
        err = rel_linf(np.asarray(g).reshape(ref.shape), ref)
        announce(f"[boundary] batch {label} problem {k} ({w.name}, n = {w.n[0]}): rel Linf vs oracle {err:.1e}")
        assert err <= TOL, (k, err)
        assert c["violations"] == 0 == st["violations"]
