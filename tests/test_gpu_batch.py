"""Batched form: independent problems of uneven sizes advanced by one launch
per kernel and stage (HIP graph per step) give the same states as the
single-problem path, problem by problem (to rounding), and match the
oracle."""
import numpy as np
import pytest

from parity_util import (_perturbed, announce, gpu_for, oracle_for, random_scalar_workload, rel_l1,
                         rel_linf, run_tol)
from paper_2509_04673_amd import workloads as W

pytestmark = pytest.mark.gpu


def _batch_for(wls, precision="fp64", **modes):
    from paper_2509_04673_amd.cem import BatchSolver
    w0 = wls[0]
    probs = [(w.d, w.p, w.n, w.lo, w.hi) for w in wls]
    b = BatchSolver(probs, w0.kind, w0.velocity, w0.gamma_gas, w_lin=w0.w_lin, q=w0.q, precision=precision,
                    **modes)
    b.upload([w.u0 for w in wls])
    if w0.kind != "euler":
        b.set_bounds()
    return b


def _singles(wls, nsteps, dt, cfl, precision="fp64", **modes):
    # the batch's float64 line passes run on the matrix cores by default
    modes.setdefault("line_kernels", 1)
    outs = []
    for w in wls:
        s = gpu_for(w, modes, precision=precision)
        for _ in range(nsteps):
            s.step(dt=dt, cfl=cfl)
        outs.append(s.download().ravel())
        s.close()
    return outs


def _multiplicity(n, p):
    c = np.where(np.arange(p * n) % p == 0, 2.0, 1.0)
    return np.multiply.outer(c, c).ravel()


# sizes straddle the switch between exact periodic line rows (n < 55 for
# Q2) and the LDS / register-blocked line kernels, up to the largest mesh of
# the batched workload (n = 256)
SIZES = [32, 40, 54, 55, 64, 97, 128, 256]


def _cm(x, m):
    """component-major view (m, N) of one problem's flat state"""
    return np.asarray(x).reshape(m, -1)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_matches_single_problems_euler(precision):
    wls = W.euler_batch(seed=3, sizes=SIZES)
    announce(f"[batch] euler {len(wls)} problems {SIZES} {precision}")
    b = _batch_for(wls, precision)
    b.step(cfl=0.5, nsteps=3)
    got = b.download()
    chk = b.check()
    b.close()
    ref = _singles(wls, 3, 0.0, 0.5, precision)
    for k, (g, r) in enumerate(zip(got, ref)):
        err = rel_linf(_cm(g, 4), _cm(r, 4))
        mass = _multiplicity(SIZES[k], wls[k].p)
        e1 = rel_l1(g, r, mass)
        announce(f"[batch] problem {k} n={SIZES[k]}: batch vs single rel Linf {err:.1e}, rel L1 {e1:.1e}")
        # the same kernel bodies, compiled into the batched wrappers (the line
        # passes with other run lengths, so other summation orders): agreement
        # to rounding (an ulp here and there);
        # in the mixed form float-sized differences grow through the limiters
        # at the quadrant discontinuities within three steps
        if precision == "fp64":
            assert err <= 1e-10, (k, err)
        else:
            assert e1 <= 1e-6 and err <= 1e-4, (k, e1, err)
        assert chk[k]["violations"] == 0 and chk[k]["rho_min"] > 0 and chk[k]["p_min"] > 0


def test_batch_matches_single_problems_kpp():
    wls = [random_scalar_workload(2, 2, (n, n + 3), kind="kpp", seed=n) for n in (20, 57, 70)]
    b = _batch_for(wls)
    b.step(dt=1e-3, nsteps=4)
    got = b.download()
    b.close()
    ref = _singles(wls, 4, 1e-3, 0.0)
    for k, (g, r) in enumerate(zip(got, ref)):
        assert rel_linf(_cm(g, 1), _cm(r, 1)) <= 1e-12, k


@pytest.mark.parametrize("elem1", [0, 1], ids=["tile", "system"])
def test_batch_small_problems_match_oracle(elem1):
    # both element pass-1 kernels of 2D Euler (the autotuner's choice)
    from paper_2509_04673_amd import cem
    wls = W.euler_batch(seed=5, sizes=[8, 11, 6])
    b = _batch_for(wls)
    cem.cem_batch_set_plan(b.b, elem1_kernel=elem1)
    b.step(cfl=0.5, nsteps=2)
    got = b.download()
    b.close()
    for k, w in enumerate(wls):
        orc = oracle_for(w)
        ref, _ = orc.run(w.u0.copy(), 2, cfl=0.5)
        floor = rel_linf(orc.run(_perturbed(w.u0), 2, cfl=0.5)[0], ref)
        err = rel_linf(_cm(got[k], 4), ref)
        announce(f"[batch] oracle problem {k} n={w.n}: rel Linf {err:.1e} (oracle 1-ulp floor {floor:.1e})")
        assert err <= run_tol(floor), (k, err, floor)


@pytest.mark.timeout(900)
def test_batch_workload_octiles_match_oracle():
    # eight problems of the 512-problem benchmark workload (seed 0) that span
    # its size range, n = 32 .. 256, with their own quadrant data: one batched
    # SSP-RK3 step (adaptive dt per problem) against the oracle, float64
    idx = W.euler_batch_octiles(0)
    wls = W.euler_batch(0, only=idx)
    assert min(w.n[0] for w in wls) == 32 and max(w.n[0] for w in wls) == 256
    announce(f"[batch] workload octiles {[(w.meta['index'], w.n[0]) for w in wls]}")
    b = _batch_for(wls)
    b.step(cfl=0.5, nsteps=1)
    got = b.download()
    chk = b.check()
    b.close()
    for k, w in enumerate(wls):
        orc = oracle_for(w)
        ref, st = orc.run(w.u0.copy(), 1, cfl=0.5)
        err = rel_linf(_cm(got[k], 4), ref)
        announce(f"[batch] octile problem {w.meta['index']} n={w.n[0]}: rel Linf vs oracle {err:.1e}")
        assert err <= 1e-12, (k, err)
        assert chk[k]["violations"] == st["violations"] == 0
        assert chk[k]["rho_min"] > 0 and chk[k]["p_min"] > 0


def test_batch_graph_replay_matches_direct():
    from paper_2509_04673_amd import cem
    wls = W.euler_batch(seed=4, sizes=[33, 60, 41])
    outs = []
    for graphs in (True, False):
        b = _batch_for(wls)
        cem.cem_batch_set_graphs(b.b, graphs)
        b.step(cfl=0.5, nsteps=2)
        b.step(cfl=0.5, nsteps=1)
        outs.append(b.download(split=False))
        b.close()
    assert np.array_equal(outs[0], outs[1])


def test_batch_autotune_keeps_state_and_results():
    wls = W.euler_batch(seed=6, sizes=[36, 70, 50, 90])
    b = _batch_for(wls)
    before = b.download(split=False)
    rep = b.autotune(cfl=0.5, steps=1)
    announce(f"[batch] autotune: {rep['best']} from {len(rep['trials'])} trials")
    # a coordinate search: every value of every knob is tried, each plan
    # once (order 2, x-line caps 4, strided tile sizes 3, pass-1 kernel 2,
    # line kernels 2)
    trials = rep["trials"]
    keys = [(t["order"], t["xlines_cap"], t["ytile_lds_bytes"], t["elem1"], t["lines"]) for t in trials]
    assert len(set(keys)) == len(keys) and 9 <= len(trials) <= 12, keys
    assert rep["best"]["ms_per_step"] > 0
    assert rep["best"]["ms_per_step"] == min(t["ms_per_step"] for t in trials)
    assert {t["order"] for t in trials} == {"input", "largest_first"}
    assert {t["xlines_cap"] for t in trials} == {512, 1024, 2048, 4096}
    assert {t["ytile_lds_bytes"] for t in trials} == {20480, 40960, 57344}
    assert {t["elem1"] for t in trials} == {"tile", "system"}
    assert {t["lines"] for t in trials} == {"matrix", "vector"}
    assert np.array_equal(b.download(split=False), before)     # state restored
    b.step(cfl=0.5, nsteps=2)
    tuned = b.download(split=False)
    b.close()
    # the same plan set explicitly gives bitwise the same states (the plan
    # is the whole of what the autotuner changes); every pass-1 kernel the
    # plans can pick is compared with the oracle on its own
    from paper_2509_04673_amd import cem
    best = rep["best"]
    ref = _batch_for(wls)
    cem.cem_batch_set_plan(ref.b, 1 if best["order"] == "largest_first" else 0, best["xlines_cap"],
                           best["ytile_lds_bytes"], 1 if best["elem1"] == "system" else 0)
    cem.cem_batch_set_line_kernels(ref.b, 1 if best["lines"] == "matrix" else 0)
    ref.step(cfl=0.5, nsteps=2)
    plain = ref.download(split=False)
    ref.close()
    assert np.array_equal(tuned, plain)


def test_batch_matches_single_problems_euler3d():
    # the 3D system passes (sensor and residual halves, pass 2) in batched form
    wls = [W.euler3d(seed=s, n=n) for s, n in ((0, 6), (1, 9), (2, 5))]
    b = _batch_for(wls)
    b.step(cfl=0.5, nsteps=2)
    got = b.download()
    chk = b.check()
    b.close()
    ref = _singles(wls, 2, 0.0, 0.5)
    for k, (g, r) in enumerate(zip(got, ref)):
        err = rel_linf(_cm(g, 5), _cm(r, 5))
        announce(f"[batch] euler3d problem {k} n={wls[k].n}: batch vs single rel Linf {err:.1e}")
        assert err <= 1e-10, (k, err)
        assert chk[k]["violations"] == 0 and chk[k]["rho_min"] > 0 and chk[k]["p_min"] > 0


@pytest.mark.parametrize("mode", ["subcell", "shrink"])
def test_batch_flux_limiter_off_matches_single(mode):
    # the flux-limiter-off variant (Sec. 4.3) through the batched launches
    wls = W.euler_batch(seed=7, sizes=[24, 57, 40])
    b = _batch_for(wls, flux_mode=mode)
    b.step(cfl=0.5, nsteps=3)
    got = b.download()
    b.close()
    ref = _singles(wls, 3, 0.0, 0.5, flux_mode=mode)
    for k, (g, r) in enumerate(zip(got, ref)):
        err = rel_linf(_cm(g, 4), _cm(r, 4))
        announce(f"[batch] {mode} problem {k}: batch vs single rel Linf {err:.1e}")
        assert err <= 1e-10, (k, err)


@pytest.mark.parametrize("elem1", [0, 1], ids=["tile", "system"])
def test_batch_plan_region_holds_many_small_problems(elem1):
    # 700 small problems: every plan entry is per problem, so the plan's
    # device region (sized at creation) is tested at its largest per-problem
    # demand, the system pass 1 with its residual half, both fused and
    # unfused assembly and all line-kernel variants
    from paper_2509_04673_amd import cem
    sizes = [6 + (k % 60) for k in range(700)]
    wls = W.euler_batch(seed=9, sizes=sizes)
    b = _batch_for(wls)
    cem.cem_batch_set_plan(b.b, 1, 512, 20480, elem1)
    b.step(cfl=0.5, nsteps=1)
    chk = b.check()
    got = b.download()
    b.close()
    announce(f"[batch] plan region: {len(wls)} problems, elem1 kernel {elem1}, one step")
    for k in (0, 1, 2, 350, 699):
        s = gpu_for(wls[k])
        s.step(cfl=0.5)
        err = rel_linf(_cm(got[k], 4), _cm(s.download(), 4))
        s.close()
        assert err <= 1e-10, (k, err)
    assert all(c["violations"] == 0 and c["rho_min"] > 0 for c in chk)


def test_batch_vector_lines_match_single_problems():
    # the batch with its float64 line passes on the vector kernels
    from paper_2509_04673_amd import cem
    wls = W.euler_batch(seed=4, sizes=[32, 55, 97, 256])
    b = _batch_for(wls)
    cem.cem_batch_set_line_kernels(b.b, 0)
    b.step(cfl=0.5, nsteps=2)
    got = b.download()
    b.close()
    ref = _singles(wls, 2, 0.0, 0.5, line_kernels=0)
    for k, (g, r) in enumerate(zip(got, ref)):
        err = rel_linf(_cm(g, 4), _cm(r, 4))
        announce(f"[batch] vector lines problem {k} n={wls[k].n[0]}: batch vs single rel Linf {err:.1e}")
        assert err <= 1e-10, (k, err)
