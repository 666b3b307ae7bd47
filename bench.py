"""Benchmark: DOF x RK-stage updates per second of the limited CG-WENO
SSP-RK3 scheme on one MI355X.

Default workload: the batched 2D Euler problem set, 512 independent
four-quadrant Riemann problems on the unit square (gamma = 1.4), Bernstein
Q2 on square meshes of n_k^2 cells, n_k = 32 + floor(225 U) drawn from a
seeded splitmix64 (seed 0: 196.8M DOFs), float64, cfl 0.5 with each
problem's own adaptive dt.  All problems advance together (one launch per
kernel and stage, each step one HIP graph, autotuned plan).  A step is one
full SSP-RK3 step (three stages, each the whole five-step algorithm:
projected gradient, WENO sensor and residual, consistent-mass solve, facet
fluxes with the flux limiter, element contributions with the slope limiter,
assembly and the RK combination).  Inputs are resident in HBM when the timed
region starts.  --workload selects the single-problem workloads (kpp2d,
euler2d, euler3d, adv1d; the non-periodic 1D lines sod1d, blast1d,
shuosher1d, inflow1d, by default Q2 on 2^20 cells) and --precision mixed the
mixed-precision form.

Prints one JSON line: the throughput (HIP events around the graph-replayed
timed region), a roofline record of the dominant kernel, the float64 oracle
timed on the host on a bounded sample of the same workload, and for the
mixed form its error against the oracle.

Roofline: the dominant kernel is the one-launch-per-stage kernel with the
largest warm-up time; its average duration comes from a pass of directly
launched steps right after the timed region, each launch carrying HIP events
that take the dispatch's own timestamps.  achieved = the algorithmic minimum
of a stage, 64/3 B per DOF-stage (stage 0 reads and writes the float64
state, stages 1-2 also read the step base), times the DOFs one launch
processes, over that duration; the same record holds the flop view (the
kernel's own flop count against the FP64 vector peak), the whole stage
against both peaks, and the HBM bytes the counters saw (per launch and per
DOF-stage of the whole stage) when the committed rocprofv3 summary of this
workload was taken on the current sources.

Profiling helpers: --copy-probe BYTES runs a plain device copy (calibration
of the byte counters) and --summarize-profile DIR writes that summary from
rocprofv3 CSV output.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_VECTOR_TFLOPS = 78.6      # MI355X FP64 vector peak
FP32_VECTOR_TFLOPS = 157.3     # MI355X FP32 vector peak (the element passes of the mixed form)
COPY_PROBE_BYTES = 1 << 28     # plain copy used to calibrate the byte counters


# per state and direction (the nonconvex flux: one branch-selected quadratic)
FLUX_FLOPS = {"advection": 1, "kpp": 40, "euler": 30, "nonconvex": 4}


def elem1_flops(d, p, m, kind, part=0):
    """Float64 operations of the element pass per element (FMA = 2), by the
    sum-factorised algorithm: cell average, WENO sensor (2d candidate
    extensions and 2d + 2 packed quadratic forms), interpolation to the
    (p+1)^d Gauss points, fluxes, gradient test, stabilisation (2 d^2
    one-axis passes), facet fluxes; transcendental fluxes at a nominal 40.
    part 1: sensor and facets only, part 2: residual only (the two launches
    of the 3D Euler pass)."""
    nl, p1 = (p + 1) ** d, p + 1
    ax = 2 * nl * p1                       # one sum-factorised axis pass
    qs = nl * (nl + 1)                     # one packed quadratic form
    weno = m * (nl + qs + 2 * d * (2 * nl + p1 * 2 * nl + qs) + 4 * d * nl + qs + 6 * (2 * d + 1))
    resid = m * (d * ax + d * d * ax) + nl * (d * FLUX_FLOPS[kind] + 2 * d) + m * (2 * d * d * ax + 4 * nl)
    facets = 2 * d * (m * (nl // p1) + 10 * m + FLUX_FLOPS[kind])
    if part == 1:
        return weno + facets + m * nl
    if part == 2:
        return resid
    return weno + resid + facets + m * nl


def split_elem1(wl):
    """The 3D Euler element pass 1 runs as two launches (sensor and facets;
    residual)."""
    return wl.kind == "euler" and wl.d == 3


def elem2_flops(d, p, m, kind):
    """Float64 operations of the limiter / contribution pass per element:
    flux limiter on 2d facets, boundary integral (2d facet Gram passes),
    consistent-mass term (d axis passes), contributions, slope limiter."""
    nl, p1 = (p + 1) ** d, p + 1
    nf = nl // p1
    return (2 * d * m * 12 + 2 * d * m * 2 * nf * p1 * max(d - 1, 1) + m * (d * 2 * nl * p1 + 10 * nl)
            + nl * (8 if m == 1 else 40) + 4 * m * nl)


def kernel_flops(name, wl, E):
    """Arithmetic of one launch of an element pass over E elements (the
    kernel's own flop count by the sum-factorised algorithm; zero for the
    streaming kernels)."""
    d, p, m = wl.d, wl.p, wl.m
    if name == "elem1":
        return E * elem1_flops(d, p, m, wl.kind, 1 if split_elem1(wl) else 0)
    if name == "elem1r":
        return E * elem1_flops(d, p, m, wl.kind, 2)
    if name == "elem2":
        return E * elem2_flops(d, p, m, wl.kind)
    return 0.0


# The algorithmic minimum HBM traffic of a stage per DOF: stage 0 reads and
# writes the float64 state (16 B), stages 1 and 2 also read the step base
# (24 B each): 64/3 B per DOF-stage over an SSP-RK3 step.
MIN_BYTES_PER_DOF_STAGE = 64.0 / 3.0
# Arithmetic of a whole stage per DOF (sum-factorised estimate, FMA = 2) per
# workload: the WENO forms, the residual contractions, the facet pass, the
# limiters and the line operators.
STAGE_FLOPS_PER_DOF = {"adv1d": 200.0, "kpp2d": 1250.0, "euler2d": 1180.0, "euler_batch": 1070.0,
                       "euler3d": 3900.0}


def source_digest():
    """sha256 of the kernel sources and build flags: counter figures taken on
    another digest no longer describe the kernels that run."""
    import hashlib
    h = hashlib.sha256()
    for f in ("csrc/kernels.hpp", "csrc/kernels_sys.hpp", "csrc/kernels_batch.hpp", "csrc/api.hip",
              "csrc/tables.cpp", "csrc/tables.hpp", "build.py"):
        with open(os.path.join(ROOT, "paper_2509_04673_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


PROFILE_DIR = os.path.join(ROOT, "profiles")


def profile_name(wl, precision="fp64"):
    tag = "" if precision == "fp64" else "_mixed"
    return f"{wl.name}_{'x'.join(str(k) for k in wl.n)}_q{wl.p}{tag}_stage_kernels.md"


def _read_csv(path):
    import csv
    with open(path) as fh:
        return list(csv.DictReader(fh))


def _one(folder, suffix):
    import glob
    hits = sorted(glob.glob(os.path.join(folder, "**", "*" + suffix), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {folder}")
    return hits[0]


def _counter_means(folder):
    """Mean counter value per kernel name and counter over the dispatches:
    {kernel: {counter: mean}}."""
    agg = {}
    for r in _read_csv(_one(folder, "counter_collection.csv")):
        agg.setdefault(r["Kernel_Name"], {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in agg.items()}


# request-size resolved HBM counters (one pass each): bytes read are the 32,
# 64 and 128 byte read requests of the L2 to memory; bytes written the 32
# and 64 byte write requests (the WRITE_SIZE definition)
RD_COUNTERS = "TCC_EA0_RDREQ_32B_sum TCC_EA0_RDREQ_64B_sum TCC_EA0_RDREQ_128B_sum TCC_EA0_RDREQ_sum"
WR_COUNTERS = "TCC_EA0_WRREQ_sum TCC_EA0_WRREQ_64B_sum"


def _read_bytes(c):
    return 32.0 * c["TCC_EA0_RDREQ_32B_sum"] + 64.0 * c["TCC_EA0_RDREQ_64B_sum"] + 128.0 * c["TCC_EA0_RDREQ_128B_sum"]


def _write_bytes(c):
    return 32.0 * (c["TCC_EA0_WRREQ_sum"] - c["TCC_EA0_WRREQ_64B_sum"]) + 64.0 * c["TCC_EA0_WRREQ_64B_sum"]


def summarize_profile(out_dir, dest, command, copy_bytes):
    """Write the rocprofv3 summary of one bench workload: kernel-trace stats
    and the HBM bytes per dispatch.  With the request-size passes (rd, wr)
    the bytes are 32/64/128 B read requests and 32/64 B write requests of
    the L2 to memory, checked on a plain device copy of copy_bytes; without
    them, FETCH_SIZE / WRITE_SIZE scaled by the factor that makes the copy
    read what it moved (the older calibration; FETCH_SIZE undercounts 128 B
    requests on gfx950, which is what that factor made up for the copy)."""
    stats = _read_csv(_one(os.path.join(out_dir, "stats"), "kernel_stats.csv"))
    resolved = os.path.isdir(os.path.join(out_dir, "rd"))
    counters = resolved or os.path.isdir(os.path.join(out_dir, "fetch"))
    per = {}            # kernel -> (read bytes, written bytes, FETCH_SIZE KiB, WRITE_SIZE KiB)
    ffac = wfac = None
    ck = None
    if resolved:
        rd, wr = _counter_means(os.path.join(out_dir, "rd")), _counter_means(os.path.join(out_dir, "wr"))
        for k in rd:
            if k in wr:
                per[k] = (_read_bytes(rd[k]), _write_bytes(wr[k]), None, None)
        crd, cwr = _counter_means(os.path.join(out_dir, "copy_rd")), _counter_means(os.path.join(out_dir, "copy_wr"))
        ck = max(crd, key=lambda k: _read_bytes(crd[k]))
        cr, cw = _read_bytes(crd[ck]), _write_bytes(cwr[ck])
        calib = (f"HBM bytes from the request-size counters ({RD_COUNTERS}; {WR_COUNTERS}): read = "
                 f"32 n32 + 64 n64 + 128 n128, written = 32 (n - n64) + 64 n64 per dispatch.  Check on a "
                 f"plain device copy of {copy_bytes} bytes (`{ck}`): read {cr:.0f} B ({cr / copy_bytes:.3f} "
                 f"of the copy), written {cw:.0f} B ({cw / copy_bytes:.3f}).")
    elif counters:
        fetch = _counter_means(os.path.join(out_dir, "fetch"))
        write = _counter_means(os.path.join(out_dir, "write"))
        cf = _counter_means(os.path.join(out_dir, "copy_fetch"))
        cwm = _counter_means(os.path.join(out_dir, "copy_write"))
        ck = max(cf, key=lambda k: cf[k]["FETCH_SIZE"])
        kib = copy_bytes / 1024.0
        ffac, wfac = kib / cf[ck]["FETCH_SIZE"], kib / cwm[ck]["WRITE_SIZE"]
        for k in fetch:
            if k in write:
                f, w = fetch[k]["FETCH_SIZE"], write[k]["WRITE_SIZE"]
                per[k] = (f * ffac * 1024.0, w * wfac * 1024.0, f, w)
        calib = (f"Counter calibration: a plain device copy of {copy_bytes} bytes (`{ck}`) reads "
                 f"FETCH_SIZE {cf[ck]['FETCH_SIZE']:.0f} KiB and WRITE_SIZE {cwm[ck]['WRITE_SIZE']:.0f} KiB "
                 f"per dispatch, so traffic = {ffac:.3f} x FETCH_SIZE + {wfac:.3f} x WRITE_SIZE.")
    else:
        calib = "Kernel trace only (no counter passes for this workload)."
    rows, data = [], {}
    for r in stats:
        name = r["Name"]
        if "cem::" not in name:
            continue
        avg_us = float(r["AverageNs"]) / 1e3
        rb, wb, f, w = per.get(name, (None, None, None, None))
        tr = None if rb is None else rb + wb
        data[name] = dict(calls=int(r["Calls"]), avg_us=avg_us, read_bytes=rb, write_bytes=wb,
                          fetch_kib=f, write_kib=w, traffic_bytes=tr)
        rows.append(f"| `{name}` | {r['Calls']} | {avg_us:.2f} | {float(r['Percentage']):.1f} | "
                    + (f"{rb / 1e6:.1f} | {wb / 1e6:.1f} | {tr / 1e6:.1f} | {tr / (avg_us * 1e-6) / 1e9:.0f} |"
                       if tr is not None else "- | - | - | - |"))
    sq_rows = []
    if os.path.isdir(os.path.join(out_dir, "sq")):
        # wave-level counters: VALU busy (% of the kernel's GPU time with a
        # VALU instruction in flight, per CU), occupancy (% of the 32 wave
        # slots of a CU, as rocprofv3's OccupancyPercent), waiting (% of wave
        # cycles a wave waited to issue), FP64 flops the VALU executed
        sq = _counter_means(os.path.join(out_dir, "sq"))
        cu, xcc = 256.0, 8.0
        for name, c in sq.items():
            if "cem::" not in name or name not in data:
                continue
            # GRBM_GUI_ACTIVE is reported summed over the 8 XCDs, each busy
            # for the whole dispatch: per-XCD active cycles = sum / 8
            g = c.get("GRBM_GUI_ACTIVE", 0.0) / xcc
            if g <= 0:
                continue
            valu = 100.0 * c["SQ_ACTIVE_INST_VALU"] / cu / g
            occ = 400.0 * c["SQ_WAVE_CYCLES"] / g / cu / 32.0
            wait = 100.0 * c["SQ_WAIT_INST_ANY"] / max(c["SQ_WAVE_CYCLES"], 1.0)
            data[name].update(valu_busy_pct=valu, occupancy_pct=occ, wait_pct=wait,
                              valu_insts=c["SQ_INSTS_VALU"], lds_insts=c["SQ_INSTS_LDS"], waves=c["SQ_WAVES"],
                              fp64_flops_counter=c["SQ_INSTS_VALU_FLOPS_FP64"])
            sq_rows.append(f"| `{name}` | {valu:.1f} | {occ:.1f} | {wait:.1f} | {c['SQ_WAVES']:.0f} | "
                           f"{c['SQ_INSTS_VALU'] / 1e6:.1f} | {c['SQ_INSTS_LDS'] / 1e6:.2f} |")
    blob = dict(digest=source_digest(), resolved=resolved, fetch_factor=ffac, write_factor=wfac,
                copy_kernel=ck, copy_bytes=copy_bytes, kernels=data)
    sq_text = ([
        "Wave counters per dispatch (SQ_ACTIVE_INST_VALU, SQ_WAVE_CYCLES, SQ_WAIT_INST_ANY, SQ_WAVES, "
        "SQ_INSTS_VALU, SQ_INSTS_LDS, GRBM_GUI_ACTIVE; 256 CUs in 8 XCDs, GRBM_GUI_ACTIVE summed over the "
        "XCDs): VALU busy = 100 ACTIVE_INST_VALU / 256 / (GUI_ACTIVE / 8) (rocprofv3's VALUBusy), "
        "occupancy = 400 WAVE_CYCLES / (GUI_ACTIVE / 8) / 256 / 32 (OccupancyPercent: % of the 32 wave "
        "slots of a CU), waiting = 100 WAIT_INST_ANY / WAVE_CYCLES (% of wave time waiting to issue).", "",
        "| kernel | VALU busy % | occupancy % | waiting % | waves | VALU Minsts | LDS Minsts |",
        "|---|---|---|---|---|---|---|", *sq_rows, ""] if sq_rows else [])
    text = ["# Stage kernels: rocprofv3 kernel trace" + (" and HBM counters" if counters else ""), "",
            "Command (from the repository root, R = its absolute path):", "", "```", command.strip(), "```", "",
            calib, "",
            "| kernel | calls | avg us | % time | read MB | written MB | traffic MB | GB/s |",
            "|---|---|---|---|---|---|---|---|", *rows, "", *sq_text,
            "Machine-readable copy (read by bench.py for the roofline traffic):", "",
            "```json", json.dumps(blob), "```", ""]
    with open(dest, "w") as fh:
        fh.write("\n".join(text))
    print(f"wrote {dest}", flush=True)


def _load_profile(fname):
    """The machine-readable blob of a committed profile summary, or None."""
    path = os.path.join(PROFILE_DIR, fname)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    try:
        return json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (IndexError, ValueError):
        return None


def _kernel_matches(name, patterns):
    """Device kernel name against the patterns of a timing id (batched
    wrappers kb_* count as their single-problem kernels k_*)."""
    base = name.replace("cem::kb_", "cem::k_")
    return any(k in base for k in patterns)


def profiled_traffic(fname, dominant, dofs):
    """From the committed counter summary (None where it is missing, holds no
    counters, or was taken on other sources): HBM bytes per launch of the
    dominant kernel, and the whole stage's HBM bytes per DOF-stage (each
    kernel's bytes per dispatch times its dispatches per stage, counted
    against the update kernel's, which runs once per stage)."""
    blob = _load_profile(fname)
    if blob is None or blob.get("digest") != source_digest() or not any(
            r.get("traffic_bytes") is not None for r in blob.get("kernels", {}).values()):
        return None, None, blob
    ks = blob["kernels"]
    upd = [r["calls"] for n, r in ks.items() if _kernel_matches(n, DEVICE_KERNELS["update"])]
    dom = [r["traffic_bytes"] for n, r in ks.items() if _kernel_matches(n, DEVICE_KERNELS[dominant])]
    per_launch = sum(dom) / len(dom) if dom else None
    stage = None
    if upd and all(r["traffic_bytes"] is not None for r in ks.values()):
        stage_calls = sum(upd)
        tot = sum(r["traffic_bytes"] * r["calls"] for n, r in ks.items() if "k_inv_partial" not in n)
        stage = tot / stage_calls / dofs
    return per_launch, stage, blob


# device kernel names behind each timing id
DEVICE_KERNELS = {"grad_line": ["k_line_multi", "k_line_x", "k_line_y", "k_line_fast", "k_line<", "k_line(",
                                "k_line_bnd"],
                  "elem1": ["k_elem1"], "gather_r": ["k_gather"],
                  "mass_line": ["k_line_y", "k_line_fast", "k_line_bnd"],
                  "elem2": ["k_elem2"], "update": ["k_update"], "elem1r": ["k_resid"],
                  "stage_dt": ["k_stage_dt"]}


def copy_probe(nbytes):
    """Plain device copy of a known size (calibrates the FETCH_SIZE and
    WRITE_SIZE counters of a profiling run against bytes actually moved)."""
    import torch
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    # the achievable HBM rate of a plain copy (read + write), for context
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(10):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    gbs = 2 * n * 8 * 10 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    print(json.dumps(dict(copy_probe_bytes=n * 8, copies=13, copy_gb_per_s=gbs)), flush=True)


def host_info():
    """CPU model and logical core count of the host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def _oracle_for(wl, method=None):
    from oracle import Mesh, Oracle, Params, Problem
    bc = getattr(wl, "bc", None)
    mesh = Mesh(wl.d, wl.p, wl.n, wl.lo, wl.hi, periodic=bc is None)
    lo, hi = float(wl.u0.min()), float(wl.u0.max())
    for kind, state in (bc or ()):
        if kind == "state" and wl.kind != "euler":
            lo, hi = min(lo, float(state[0])), max(hi, float(state[0]))
    prob = Problem(mesh, wl.kind, wl.velocity, wl.gamma_gas, params=Params(w_lin=wl.w_lin, q=wl.q, **(method or {})),
                   u_min=lo, u_max=hi, bc=bc)
    return Oracle(prob)


def _oracle_stages(wl, seconds, max_stages=None, method=None):
    """Whole forward-Euler stages of the oracle on one workload, one thread,
    until `seconds` have elapsed (at least one): (stages, elapsed s)."""
    from threadpoolctl import threadpool_limits
    from oracle import CFLViolation
    with threadpool_limits(limits=1):
        orc = _oracle_for(wl, method)
        dt = wl.dt if wl.dt > 0 else wl.cfl * orc.max_dt(wl.u0)
        u = wl.u0.copy()
        stages = 0
        t0 = time.perf_counter()
        while True:
            try:
                u, _ = orc.fe_stage(u, dt)
            except CFLViolation:
                # the waves sped up: a new step size from the current state
                # (its evaluation is not counted as oracle work)
                t1 = time.perf_counter()
                dt = wl.cfl * orc.max_dt(u)
                t0 += time.perf_counter() - t1
                continue
            stages += 1
            el = time.perf_counter() - t0
            if el >= seconds or (max_stages and stages >= max_stages):
                return stages, el


def _oracle_stage_job(wl):
    """One oracle stage of one problem (a worker of the all-core run)."""
    st, el = _oracle_stages(wl, 0.0, 1)
    return wl.dofs * st, el


def cpu_baseline(wls, seconds, label, all_cores=False, method=None):
    """The float64 oracle timed on the host: one thread on whole stages of
    the sample workloads (in turn, until `seconds` have elapsed); with
    all_cores, also one stage of every sample problem at once in a pool of
    single-threaded processes (one per core, at most one per problem)."""
    model, ncpu = host_info()
    dof_stages, el = 0, 0.0
    per = max(seconds / len(wls), 1e-3)
    for w in wls:
        st, e = _oracle_stages(w, per, method=method)
        dof_stages += w.dofs * st
        el += e
    out = dict(value=dof_stages / el, unit="DOF*stage/s", cores=1, kind="oracle",
               sample=f"{label}: {dof_stages} DOF-stages of forward-Euler stages, numpy float64, "
                      f"1 thread, {el:.1f} s", cpu_model=model, host_cores=ncpu)
    if all_cores and len(wls) > 1:
        import multiprocessing as mp
        workers = max(1, min(len(wls), ncpu or 1, 16))
        ctx = mp.get_context("fork")
        t0 = time.perf_counter()
        with ctx.Pool(workers) as pool:
            res = pool.map(_oracle_stage_job, wls)
        wall = time.perf_counter() - t0
        out["all_cores"] = dict(value=sum(r[0] for r in res) / wall, cores=workers,
                                sample=f"one stage of each of the {len(wls)} sample problems, "
                                       f"{workers} single-threaded processes, {wall:.1f} s wall")
    return out


def mixed_error(make_gpu_run, wls, nsteps=1, method=None):
    """Relative L1 error per component (lumped masses) of the mixed form
    against the float64 oracle after nsteps SSP-RK3 steps, max over
    components and sample problems; make_gpu_run(wls, nsteps) returns the
    GPU states (one (m, N) array per workload)."""
    import numpy as np
    got = make_gpu_run(wls, nsteps)
    worst = 0.0
    for w, g in zip(wls, got):
        orc = _oracle_for(w, method)
        ref, _ = orc.run(w.u0.copy(), nsteps, dt=(w.dt if w.dt > 0 else None), cfl=w.cfl)
        mass = orc.mesh.multiplicity() * orc.mesh.h ** orc.mesh.d / orc.mesh.nloc
        g = np.asarray(g).reshape(ref.shape)
        num = np.sum(mass * np.abs(g - ref), axis=1)
        den = np.sum(mass * np.abs(ref), axis=1)
        worst = max(worst, float(np.max(num / np.where(den > 0, den, 1.0))))
    return worst


def roofline_record(dominant, kt, wl, dofs, E, value, mixed, profile_file):
    """The roofline record of the dominant kernel (see the module docstring)."""
    kms, kcnt = kt[dominant]
    avg_s = (kms / kcnt) * 1e-3 if kcnt else float("nan")
    nbytes = MIN_BYTES_PER_DOF_STAGE * dofs
    achieved = nbytes / avg_s / 1e9
    kfl = kernel_flops(dominant, wl, E)
    fpeak = FP32_VECTOR_TFLOPS if mixed else FP64_VECTOR_TFLOPS
    traffic, stage_traffic, prof = profiled_traffic(profile_file, dominant, dofs)
    prof_us = None
    if prof is not None and traffic is not None:
        us = [r["avg_us"] for n, r in prof["kernels"].items() if _kernel_matches(n, DEVICE_KERNELS[dominant])]
        prof_us = sum(us) / len(us) if us else None
    sflops = STAGE_FLOPS_PER_DOF.get(wl.name)
    return dict(
        bound="hbm", kernel=dominant, achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
        frac=achieved / HBM_PEAK_GBS, traffic=traffic,
        algorithmic_bytes=nbytes, min_bytes_per_dof_stage=MIN_BYTES_PER_DOF_STAGE, dofs_per_launch=dofs,
        avg_launch_us=avg_s * 1e6, launches=kcnt, profiled_avg_us=prof_us,
        traffic_per_dof_stage_kernel=None if traffic is None else traffic / dofs,
        traffic_per_dof_stage_stage=stage_traffic,
        flop_view=dict(kernel_flops=kfl, achieved=kfl / avg_s / 1e12, peak=fpeak, unit="TFLOP/s",
                       frac=kfl / avg_s / 1e12 / fpeak),
        stage_view=dict(hbm_frac=MIN_BYTES_PER_DOF_STAGE * value / (HBM_PEAK_GBS * 1e9),
                        flops_per_dof_stage=sflops,
                        alu_frac=None if sflops is None else sflops * value / (fpeak * 1e12)))


def _dominant(warm, nwarm):
    """The one-launch-per-stage kernel with the largest warm-up time."""
    single = {k: v for k, v in warm.items() if v[1] == 3 * nwarm}
    return max(single, key=lambda k: single[k][0])


def bench_batch(args):
    """The batched workload: count independent four-quadrant Euler problems
    (Q2, n_k^2 meshes, n_k = 32 + floor(225 U)) advanced together, one launch
    per kernel and stage, each step one HIP graph; adaptive dt per problem."""
    import numpy as np
    import torch
    from paper_2509_04673_amd import cem, workloads
    prec = args.precision
    mixed = prec == "mixed"
    wls = workloads.euler_batch(seed=0, count=args.count)
    dofs = sum(w.dofs for w in wls)
    E = sum(w.n[0] * w.n[1] for w in wls)
    print(f"[bench] batched Euler: {len(wls)} problems, n in [{min(w.n[0] for w in wls)}, "
          f"{max(w.n[0] for w in wls)}], {dofs} DOFs, precision={prec}", flush=True)
    dev = torch.device("cuda:0")
    b = cem.BatchSolver([(w.d, w.p, w.n, w.lo, w.hi) for w in wls], "euler", gamma_gas=wls[0].gamma_gas,
                        w_lin=wls[0].w_lin, precision=prec)
    b.upload([w.u0 for w in wls])
    wl0 = wls[0]
    del wls
    cfl = 0.5
    if args.plan:
        vals = [int(v) for v in args.plan.split(",")]
        o, xc, yc, e1 = vals[:4]
        lines = vals[4] if len(vals) > 4 else 1
        cem.cem_batch_set_plan(b.b, o, xc, yc, e1)
        cem.cem_batch_set_line_kernels(b.b, lines)
        tune = dict(best=dict(order=o, xlines_cap=xc, ytile_lds_bytes=yc, elem1=e1, lines=lines, source="--plan"),
                    trials=[])
    elif args.no_autotune:
        tune = dict(best=None, trials=[])
    else:
        tune = b.autotune(cfl=cfl, steps=1)
    print(f"[bench] autotuned plan: {tune['best']} ({len(tune['trials'])} plans tried)", flush=True)
    for t in tune["trials"]:
        print(f"[bench]   trial {t}", flush=True)

    nwarm = max(1, args.warmup)
    cem.cem_batch_set_timing(b.b, (1 << len(cem.KERNELS)) - 1)
    b.step(cfl=cfl, nsteps=nwarm)
    warm = cem.cem_batch_kernel_times(b.b)
    dominant = _dominant(warm, nwarm)
    kernel_ms_per_step = sum(v[0] for v in warm.values()) / nwarm
    print("[bench] warm-up kernel ms: " + ", ".join(f"{k}={v[0]:.2f}/{v[1]}" for k, v in warm.items()
                                                   if v[1]), flush=True)
    cem.cem_batch_set_timing(b.b, 0)
    b.step(cfl=cfl, nsteps=1)                  # captures the graph
    cem.cem_batch_reset_counters(b.b)
    stream = b.stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(dev)
    w0 = time.perf_counter()
    ev0.record(stream)
    b.step(cfl=cfl, nsteps=args.steps)
    ev1.record(stream)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - w0
    ms = ev0.elapsed_time(ev1)
    chk = b.check()

    nroof = max(1, min(args.steps, 10))
    cem.cem_batch_set_timing(b.b, 1 << cem.KERNELS.index(dominant))
    b.step(cfl=cfl, nsteps=nroof)
    kt = cem.cem_batch_kernel_times(b.b)
    cem.cem_batch_set_timing(b.b, 0)
    b.close()
    del b
    torch.cuda.empty_cache()

    value = dofs * 3 * args.steps / (ms * 1e-3)
    wlb = workloads.Workload("euler_batch", 2, 2, (args.count,), (0.0, 0.0), (1.0, 1.0), "euler",
                             np.zeros((4, 1)))
    pname = f"euler_batch_{args.count}_q2{'_mixed' if mixed else ''}_stage_kernels.md"
    roof = roofline_record(dominant, kt, wlb, dofs, E, value, mixed, pname)

    # the oracle and the mixed-form error on eight problems spanning the sizes
    sample = workloads.euler_batch(0, count=args.count, only=workloads.euler_batch_octiles(0, args.count))
    label = f"the 8 problems at the size octiles (n = {', '.join(str(w.n[0]) for w in sample)})"
    cpu, err = None, None
    if not args.no_cpu_baseline:
        print(f"[bench] timing the oracle for ~{args.cpu_seconds:.0f} s on {label}", flush=True)
        cpu = cpu_baseline(sample, args.cpu_seconds, label, all_cores=True)
        cpu["extrapolated_full_batch_s_per_stage"] = dofs / cpu["value"]
    if mixed and not args.no_error:
        def run(ws, nsteps):
            bb = cem.BatchSolver([(w.d, w.p, w.n, w.lo, w.hi) for w in ws], "euler",
                                 gamma_gas=ws[0].gamma_gas, w_lin=ws[0].w_lin, precision="mixed")
            bb.upload([w.u0 for w in ws])
            bb.step(cfl=cfl, nsteps=nsteps)
            out = bb.download()
            bb.close()
            return out
        print("[bench] mixed-form error against the oracle (1 step, 8 problems)", flush=True)
        err = dict(rel_l1=mixed_error(run, sample, 1), sample=f"{label}, one SSP-RK3 step, max over "
                                                                "components and problems")
    out = dict(metric="DOF*RK-stage updates/s", value=value, unit="DOF*stage/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=ms / args.steps,
               higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f32+f64" if mixed else "f64", data="synthetic",
               config=dict(workload="euler_batch", problems=args.count, dim=2, degree=2, dofs=dofs,
                           elements=E, physics="euler", cfl=cfl, seed=0, precision=prec, wall_s=wall,
                           violations=int(sum(c["violations"] for c in chk)),
                           rho_min=min(c["rho_min"] for c in chk), p_min=min(c["p_min"] for c in chk),
                           autotune=tune["best"], autotune_trials=len(tune["trials"]),
                           # what one launch per kernel costs: the graph's time per step against
                           # the sum of the kernels' own durations (dispatch timestamps)
                           launch_gap=dict(kernel_ms_per_step=kernel_ms_per_step,
                                           graph_ms_per_step=ms / args.steps,
                                           gap_frac=(ms / args.steps - kernel_ms_per_step) / (ms / args.steps))),
               roofline=roof, cpu_baseline=cpu)
    if err is not None:
        out["mixed_error"] = err
    print(json.dumps(out), flush=True)


def bench_line_batch(args):
    """Many independent Euler lines (the paper's modified Sod, blast and
    Shu-Osher problems, Q2 by default, 64..512 cells each, their own
    boundary data) advanced together by the batched form: one launch per
    kernel and stage, each step one HIP graph, adaptive dt per problem."""
    import torch
    from paper_2509_04673_amd import cem, workloads
    p = args.degree or 2
    wls = workloads.line_batch(seed=0, count=args.count, p=p)
    dofs = sum(w.dofs for w in wls)
    E = sum(w.n[0] for w in wls)
    print(f"[bench] batched lines: {len(wls)} problems, n in [{min(w.n[0] for w in wls)}, "
          f"{max(w.n[0] for w in wls)}], {dofs} DOFs", flush=True)
    dev = torch.device("cuda:0")
    b = cem.BatchSolver([(w.d, w.p, w.n, w.lo, w.hi, w.bc) for w in wls], "euler", gamma_gas=wls[0].gamma_gas,
                        w_lin=wls[0].w_lin)
    b.upload([w.u0 for w in wls])
    cfl = 0.5
    nwarm = max(1, args.warmup)
    cem.cem_batch_set_timing(b.b, (1 << len(cem.KERNELS)) - 1)
    b.step(cfl=cfl, nsteps=nwarm)
    warm = cem.cem_batch_kernel_times(b.b)
    dominant = _dominant(warm, nwarm)
    print("[bench] warm-up kernel ms: " + ", ".join(f"{k}={v[0]:.2f}/{v[1]}" for k, v in warm.items()
                                                   if v[1]), flush=True)
    cem.cem_batch_set_timing(b.b, 0)
    b.step(cfl=cfl, nsteps=1)                  # captures the graph
    cem.cem_batch_reset_counters(b.b)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(dev)
    w0 = time.perf_counter()
    ev0.record(b.stream)
    b.step(cfl=cfl, nsteps=args.steps)
    ev1.record(b.stream)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - w0
    ms = ev0.elapsed_time(ev1)
    chk = b.check()
    cem.cem_batch_set_timing(b.b, 1 << cem.KERNELS.index(dominant))
    b.step(cfl=cfl, nsteps=max(1, min(args.steps, 10)))
    kt = cem.cem_batch_kernel_times(b.b)
    cem.cem_batch_set_timing(b.b, 0)
    b.close()
    value = dofs * 3 * args.steps / (ms * 1e-3)
    wlb = workloads.Workload("line_batch", 1, p, (args.count,), (0.0,), (1.0,), "euler", wls[0].u0[:, :1])
    pname = f"line_batch_{args.count}_q{p}_stage_kernels.md"
    roof = roofline_record(dominant, kt, wlb, dofs, E, value, False, pname)
    # the oracle on one problem of each kind at the smallest, middle and
    # largest size of the batch
    order = sorted(range(len(wls)), key=lambda k: wls[k].n[0])
    pick = []
    for kind in range(3):
        ks = [k for k in order if k % 3 == kind]
        pick.append(ks[[0, len(ks) // 2, -1][kind]])
    sample = [wls[k] for k in pick]
    label = "one Sod, blast and Shu-Osher line of the batch (n = " + ", ".join(str(w.n[0]) for w in sample) + ")"
    cpu = None
    if not args.no_cpu_baseline:
        print(f"[bench] timing the oracle for ~{args.cpu_seconds:.0f} s on {label}", flush=True)
        cpu = cpu_baseline(sample, args.cpu_seconds, label)
        cpu["extrapolated_full_batch_s_per_stage"] = dofs / cpu["value"]
    out = dict(metric="DOF*RK-stage updates/s", value=value, unit="DOF*stage/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=ms / args.steps,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
               config=dict(workload="line_batch", problems=args.count, dim=1, degree=p, dofs=dofs, elements=E,
                           physics="euler", boundary="state / wall / outflow by problem", cfl=cfl, seed=0,
                           precision="fp64", wall_s=wall, violations=int(sum(c["violations"] for c in chk)),
                           rho_min=min(c["rho_min"] for c in chk), p_min=min(c["p_min"] for c in chk)),
               roofline=roof, cpu_baseline=cpu)
    print(json.dumps(out), flush=True)


# oracle samples of the single-problem workloads: the mesh of the error and
# baseline runs where the full mesh would take the oracle minutes per stage
SAMPLE_N = {"euler2d": 256, "euler3d": 32}
# non-periodic lines: the timed size (Q2, 2^20 cells) and the oracle's sample
# (Q2, 1000 cells: its dense line solves grow with the square of the nodes)
LINE_WORKLOADS = ("sod1d", "blast1d", "shuosher1d", "inflow1d", "nonconvex1d")
LINE_BENCH = dict(n=1 << 20, p=2)
LINE_SAMPLE = dict(n=1000, p=2)


def bench_single(args):
    import numpy as np  # noqa: F401
    import torch
    from paper_2509_04673_amd import cem, workloads
    line = args.workload in LINE_WORKLOADS
    kw = {} if args.n is None else dict(n=args.n)
    if args.degree is not None:
        kw["p"] = args.degree
    if line:
        kw = dict(LINE_BENCH, **kw)
    wl = workloads.make(args.workload, seed=0, **kw)
    mixed = args.precision == "mixed"
    print(f"[bench] workload {wl.name} d={wl.d} p={wl.p} n={wl.n} dofs={wl.dofs} "
          f"precision={args.precision}", flush=True)
    dev = torch.device("cuda:0")
    method = dict(bounds=args.bounds, contrib=args.contrib)
    s = cem.Solver.from_workload(wl, device="cuda:0", precision=args.precision, **method)
    s.upload(wl.u0)
    if wl.kind != "euler":
        s.set_bounds()
    dt, cfl = (wl.dt, 0.0) if wl.dt > 0 else (0.0, wl.cfl)

    nwarm = max(1, args.warmup)
    cem.cem_set_timing(s.ctx, (1 << len(cem.KERNELS)) - 1)
    for _ in range(nwarm):
        s.step(dt, cfl)
    warm = cem.cem_kernel_times(s.ctx)
    dominant = _dominant(warm, nwarm)
    print("[bench] warm-up kernel ms: " + ", ".join(f"{k}={v[0]:.2f}/{v[1]}" for k, v in warm.items()
                                                   if v[1]), flush=True)
    cem.cem_set_timing(s.ctx, 0)
    s.step(dt, cfl)                       # captures the graph
    cem.cem_reset_counters(s.ctx)
    stream = torch.cuda.current_stream(dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(dev)
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        s.step(dt, cfl)
    ev1.record(stream)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - w0
    ms = ev0.elapsed_time(ev1)
    chk = s.check()

    nroof = min(args.steps, 50)
    cem.cem_set_timing(s.ctx, 1 << cem.KERNELS.index(dominant))
    for _ in range(nroof):
        s.step(dt, cfl)
    kt = cem.cem_kernel_times(s.ctx)
    cem.cem_set_timing(s.ctx, 0)
    E, N = s.E, s.N
    s.close()

    value = wl.dofs * 3 * args.steps / (ms * 1e-3)
    roof = roofline_record(dominant, kt, wl, wl.dofs, E, value, mixed, profile_name(wl, args.precision))

    sn = SAMPLE_N.get(wl.name) if args.n is None else None
    swl = workloads.make(args.workload, seed=0, n=sn) if sn else wl
    if line:
        sn = LINE_SAMPLE["n"]
        swl = workloads.make(args.workload, seed=0, **LINE_SAMPLE)
    label = f"the {wl.name} workload" + (f" at n = {sn}" if sn else "") + f" ({swl.dofs} DOFs)"
    cpu, err = None, None
    if not args.no_cpu_baseline:
        print(f"[bench] timing the oracle for ~{args.cpu_seconds:.0f} s on {label}", flush=True)
        cpu = cpu_baseline([swl], args.cpu_seconds, label, method=method)
    if mixed and not args.no_error:
        def run(ws, nsteps):
            outs = []
            for w in ws:
                ss = cem.Solver.from_workload(w, device="cuda:0", precision="mixed", **method)
                ss.upload(w.u0)
                if w.kind != "euler":
                    ss.set_bounds()
                for _ in range(nsteps):
                    ss.step(w.dt if w.dt > 0 else 0.0, 0.0 if w.dt > 0 else w.cfl)
                outs.append(ss.download())
                ss.close()
            return outs
        print(f"[bench] mixed-form error against the oracle (1 step, {label})", flush=True)
        err = dict(rel_l1=mixed_error(run, [swl], 1, method=method), sample=f"{label}, one SSP-RK3 step, max over components")
    out = dict(metric="DOF*RK-stage updates/s", value=value, unit="DOF*stage/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=ms / args.steps,
               higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f32+f64" if mixed else "f64", data="synthetic",
               config=dict(workload=wl.name, dim=wl.d, degree=wl.p, cells=list(wl.n),
                           boundary=None if wl.bc is None else [b[0] for b in wl.bc],
                           dofs=wl.dofs, elements=E, physics=wl.kind, dt=wl.dt if wl.dt > 0 else None,
                           cfl=None if wl.dt > 0 else wl.cfl, seed=0, precision=args.precision,
                           bounds=args.bounds, contrib=args.contrib,
                           wall_s=wall, violations=chk["violations"], clamped=chk["clamped"]),
               roofline=roof, cpu_baseline=cpu)
    if err is not None:
        out["mixed_error"] = err
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="euler_batch",
                    choices=["euler_batch", "line_batch", "kpp2d", "adv1d", "euler2d", "euler3d", "sod1d",
                             "blast1d", "shuosher1d", "inflow1d", "nonconvex1d"])
    ap.add_argument("--bounds", default="global", choices=["global", "local"],
                    help="single workloads: global or local bounds of the scalar limiters")
    ap.add_argument("--contrib", default="aec", choices=["aec", "q1"],
                    help="single workloads: element contributions of eq. (45) or their Q1 form (p = 1)")
    ap.add_argument("--count", type=int, default=None,
                    help="problems of the batched workload (euler_batch 512, line_batch 4096)")
    ap.add_argument("--n", type=int, default=None, help="cells per axis (default: workload size)")
    ap.add_argument("--degree", type=int, default=None, help="single workloads: Bernstein degree p")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="fp64, or mixed: float contractions with float64 state, limiters and dt")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-error", action="store_true", help="skip the mixed-form error run")
    ap.add_argument("--no-autotune", action="store_true", help="batched workload: default plan")
    ap.add_argument("--plan", default="", metavar="ORDER,XCAP,YTILE,ELEM1[,LINES]",
                    help="batched workload: this plan instead of the autotuner (cem_batch_set_plan; "
                         "LINES 1 matrix-core line tiles (default), 0 vector, cem_batch_set_line_kernels)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration)")
    ap.add_argument("--summarize-profile", metavar="DIR",
                    help="write the rocprofv3 summary of DIR/{stats,fetch,write,copy_fetch,copy_write}")
    ap.add_argument("--profile-command", default="", help="command text recorded in the summary")
    args = ap.parse_args()
    if args.count is None:
        args.count = 4096 if args.workload == "line_batch" else 512
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.summarize_profile:
        from paper_2509_04673_amd import workloads
        kw = {} if args.n is None else dict(n=args.n)
        if args.workload == "euler_batch":
            name = f"euler_batch_{args.count}_q2{'_mixed' if args.precision == 'mixed' else ''}_stage_kernels.md"
        elif args.workload == "line_batch":
            name = f"line_batch_{args.count}_q{args.degree or 2}_stage_kernels.md"
        else:
            if args.workload in LINE_WORKLOADS:
                kw = dict(LINE_BENCH, **kw)
            name = profile_name(workloads.make(args.workload, seed=0, **kw), args.precision)
        summarize_profile(args.summarize_profile, os.path.join(PROFILE_DIR, name),
                          args.profile_command, COPY_PROBE_BYTES)
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): this build measures "
              "the path on a single MI355X; the multi-GPU decomposition is described, not "
              "implemented", file=sys.stderr)
        sys.exit(2)
    if args.workload == "euler_batch":
        bench_batch(args)
    elif args.workload == "line_batch":
        bench_line_batch(args)
    else:
        bench_single(args)


if __name__ == "__main__":
    main()
