"""Benchmark: DOF x RK-stage updates per second of the limited CG-WENO
SSP-RK3 scheme on one MI355X.

Default workload: the 2D KPP problem (flux (sin u, cos u)) on
[-2,2]x[-2.5,1.5] with 256x256 Bernstein Q2 cells (262144 unique DOFs),
float64, fixed dt = 5e-4, seeded disc data.  A step is one full SSP-RK3 step
(three stages, each the whole five-step algorithm: projected gradient, WENO
sensor and residual, consistent-mass solve, facet fluxes with the flux
limiter, element contributions with the slope limiter, assembly and the RK
combination).  Inputs are resident in HBM when the timed region starts.

Prints one JSON line with the throughput (HIP events around the
graph-replayed timed region), a roofline record of the dominant kernel and
the float64 oracle timed on the host on a bounded sample of the same
workload.  The dominant kernel is the single-launch-per-stage kernel with the
largest warm-up time; its average duration is measured in a pass of directly
launched steps right after the timed region, each launch carrying HIP events
that take the dispatch's own timestamps.  Its achieved rate is its
algorithmic bytes (or flops, whichever bound is higher) per launch over that
duration; `traffic` is the HBM bytes per launch from the committed rocprofv3
counter summary of this workload, null when the kernel sources changed since.

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


FLUX_FLOPS = {"advection": 1, "kpp": 40, "euler": 30}   # per state and direction


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


def kernel_work(name, wl, N, E, m, mixed=False):
    """Algorithmic (bytes, flops) of one launch of a stage kernel.

    Bytes are the arrays the method must read and write in that pass, each
    once: the line operators read and write one nodal array (16 m N); the
    gather reads the element vectors and writes r and the first line pass;
    the update reads the element vectors, u and u_base and writes u (and the
    nodal fluxes of KPP).  The element passes read the nodal arrays they
    need (u, g, nodal fluxes, udot) and write the element data of the next
    pass.  In the mixed form g, r, udot and the residual vectors are float
    (4 bytes).  Flops of the line operators are those of a banded solve
    (about 8p per node, not the wider truncated-inverse apply that runs);
    those of the element passes come from elem1_flops / elem2_flops."""
    d, p = wl.d, wl.p
    nl = (p + 1) ** d
    kn = d * m * N if wl.kind == "kpp" else 0        # nodal fluxes of KPP
    f8, fr = 8.0, (4.0 if mixed else 8.0)             # state / intermediates
    if name == "grad_line":
        return m * N * (f8 + fr), 8 * p * m * N
    if name == "mass_line":
        return 2 * m * N * fr, 8 * p * m * N
    if name == "gather_r":
        return (m * nl * E + 2 * m * N) * fr, m * nl * E
    if name == "update":
        return (m * nl * E + 3 * m * N + kn) * f8, (nl + 4) * m * N
    if name == "elem1" and split_elem1(wl):
        # sensor and facets: u in; averages, low-order averages, f^A, dt_e,
        # gamma_e, nu_e out
        return m * N * f8 + (d * m + 3 + 2 * m) * E * f8, E * elem1_flops(d, p, m, wl.kind, 1)
    if name == "elem1r":
        # residual: u, g, averages, gamma_e, nu_e in; element vectors out
        rd = m * N * f8 + d * m * N * fr + (m + 2) * E * f8
        return rd + m * nl * E * fr, E * elem1_flops(d, p, m, wl.kind, 2)
    if name == "elem1":
        rd = (m * N + kn) * f8 + d * m * N * fr
        wr = m * nl * E * fr + (d * m + 3 + 2 * m) * E * f8
        return rd + wr, E * elem1_flops(d, p, m, wl.kind)
    if name == "elem2":
        rd = (m * N + kn + (d * m + 2 * m + 1) * E) * f8 + (m * N + m * nl * E) * fr
        return rd + (m * nl + m + 1) * E * f8, E * elem2_flops(d, p, m, wl.kind)
    return 0.0, 0.0


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
    """Mean counter value (KiB) per kernel name over its dispatches."""
    agg = {}
    for r in _read_csv(_one(folder, "counter_collection.csv")):
        agg.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in agg.items()}


def summarize_profile(out_dir, dest, command, copy_bytes):
    """Write the rocprofv3 summary of one bench workload: kernel-trace stats
    and FETCH_SIZE / WRITE_SIZE per dispatch, the counters scaled by the
    factor that makes a plain copy of copy_bytes read what it moved."""
    stats = _read_csv(_one(os.path.join(out_dir, "stats"), "kernel_stats.csv"))
    counters = os.path.isdir(os.path.join(out_dir, "fetch"))   # else a kernel trace only
    fetch = _counter_means(os.path.join(out_dir, "fetch")) if counters else {}
    write = _counter_means(os.path.join(out_dir, "write")) if counters else {}
    if counters:
        cf = _counter_means(os.path.join(out_dir, "copy_fetch"))
        cw = _counter_means(os.path.join(out_dir, "copy_write"))
        ck = max(cf, key=cf.get)
        kib = copy_bytes / 1024.0
        ffac, wfac = kib / cf[ck], kib / cw[ck]
    else:
        ck, ffac, wfac = None, None, None
    rows, data = [], {}
    for r in stats:
        name = r["Name"]
        if "cem::" not in name:
            continue
        avg_us = float(r["AverageNs"]) / 1e3
        f = fetch.get(name)
        w = write.get(name)
        tr = None if f is None or w is None else (f * ffac + w * wfac) * 1024.0
        data[name] = dict(calls=int(r["Calls"]), avg_us=avg_us, fetch_kib=f, write_kib=w, traffic_bytes=tr)
        rows.append(f"| `{name}` | {r['Calls']} | {avg_us:.2f} | {float(r['Percentage']):.1f} | "
                    + (f"{f:.0f} | {w:.0f} | {tr / 1e6:.2f} |" if tr is not None else "- | - | - |"))
    blob = dict(digest=source_digest(), fetch_factor=ffac, write_factor=wfac, copy_kernel=ck,
                copy_bytes=copy_bytes, kernels=data)
    calib = (f"Counter calibration: a plain device copy of {copy_bytes} bytes (`{ck}`) reads "
             f"FETCH_SIZE {cf[ck]:.0f} KiB and WRITE_SIZE {cw[ck]:.0f} KiB per dispatch, so traffic = "
             f"{ffac:.3f} x FETCH_SIZE + {wfac:.3f} x WRITE_SIZE." if counters
             else "Kernel trace only (no counter passes for this workload).")
    text = ["# Stage kernels: rocprofv3 kernel trace" + (" and HBM counters" if counters else ""), "",
            "Command (from the repository root, R = its absolute path):", "", "```", command.strip(), "```", "",
            calib, "",
            "| kernel | calls | avg us | % time | FETCH_SIZE KiB | WRITE_SIZE KiB | traffic MB |",
            "|---|---|---|---|---|---|---|", *rows, "",
            "Machine-readable copy (read by bench.py for the roofline traffic):", "",
            "```json", json.dumps(blob), "```", ""]
    with open(dest, "w") as fh:
        fh.write("\n".join(text))
    print(f"wrote {dest}", flush=True)


def profiled_traffic(wl, kernel_names, precision="fp64"):
    """Bytes per launch of the dominant kernel from the committed counter
    summary, or None when it is missing or was taken on other sources."""
    path = os.path.join(PROFILE_DIR, profile_name(wl, precision))
    if not os.path.exists(path):
        return None, None
    text = open(path).read()
    try:
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (IndexError, ValueError):
        return None, None
    if blob.get("digest") != source_digest():
        return None, blob
    for name, rec in blob["kernels"].items():
        if any(k in name for k in kernel_names):
            return rec["traffic_bytes"], blob
    return None, blob


# device kernel names behind each timing id
DEVICE_KERNELS = {"grad_line": ["k_line_multi", "k_line_x", "k_line_y", "k_line_fast", "k_line("],
                  "elem1": ["k_elem1"], "gather_r": ["k_gather"], "mass_line": ["k_line_y", "k_line_fast"],
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


def cpu_baseline(wl, seconds):
    """The float64 oracle timed on the host on whole forward-Euler stages of
    the same workload until `seconds` have elapsed (at least one stage)."""
    from threadpoolctl import threadpool_limits
    from oracle import Mesh, Oracle, Params, Problem
    mesh = Mesh(wl.d, wl.p, wl.n, wl.lo, wl.hi)
    prob = Problem(mesh, wl.kind, wl.velocity, wl.gamma_gas, params=Params(w_lin=wl.w_lin, q=wl.q),
                   u_min=float(wl.u0.min()), u_max=float(wl.u0.max()))
    with threadpool_limits(limits=1):
        orc = Oracle(prob)
        dt = wl.dt if wl.dt > 0 else wl.cfl * orc.max_dt(wl.u0)
        u = wl.u0.copy()
        stages = 0
        t0 = time.perf_counter()
        while True:
            u, _ = orc.fe_stage(u, dt)
            stages += 1
            el = time.perf_counter() - t0
            if el >= seconds:
                break
    return dict(value=wl.dofs * stages / el, unit="DOF*stage/s", cores=1, kind="oracle",
                sample=f"{stages} forward-Euler stages of the full {wl.name} workload "
                       f"({wl.dofs} DOFs), numpy float64, 1 thread, {el:.1f} s")


def bench_batch(args):
    """The batched workload: count independent four-quadrant Euler problems
    (Q2, n_k^2 meshes, n_k = 32 + floor(225 U)) advanced together, one launch
    per kernel and stage, each step one HIP graph; adaptive dt per problem."""
    import torch
    from paper_2509_04673_amd import cem, workloads
    prec = args.precision if args.precision != "fp64" or "--precision" in sys.argv else "mixed"
    wls = workloads.euler_batch(seed=0, count=args.count)
    dofs = sum(w.dofs for w in wls)
    print(f"[bench] batched Euler: {len(wls)} problems, n in [{min(w.n[0] for w in wls)}, "
          f"{max(w.n[0] for w in wls)}], {dofs} DOFs, precision={prec}", flush=True)
    dev = torch.device("cuda:0")
    b = cem.BatchSolver([(w.d, w.p, w.n, w.lo, w.hi) for w in wls], "euler", gamma_gas=wls[0].gamma_gas,
                        w_lin=wls[0].w_lin, precision=prec)
    b.upload([w.u0 for w in wls])
    del wls
    cfl = 0.5
    tune = b.autotune(cfl=cfl, steps=1)
    print(f"[bench] autotuned plan: {tune['best']}", flush=True)
    b.step(cfl=cfl, nsteps=args.warmup)
    cem.cem_batch_reset_counters(b.b)
    stream = torch.cuda.current_stream(dev)
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
    b.close()
    value = dofs * 3 * args.steps / (ms * 1e-3)
    out = dict(metric="DOF*RK-stage updates/s", value=value, unit="DOF*stage/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=ms / args.steps,
               higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f64" if prec == "fp64" else "f32+f64", data="synthetic",
               config=dict(workload="euler_batch", problems=args.count, degree=2, dofs=dofs, physics="euler",
                           cfl=cfl, seed=0, wall_s=wall,
                           violations=int(sum(c["violations"] for c in chk)),
                           rho_min=min(c["rho_min"] for c in chk), p_min=min(c["p_min"] for c in chk),
                           autotune=tune["best"]),
               roofline=None, cpu_baseline=None)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="kpp2d", choices=["kpp2d", "adv1d", "euler2d", "euler3d", "euler_batch"])
    ap.add_argument("--count", type=int, default=512, help="problems of the batched workload")
    ap.add_argument("--n", type=int, default=None, help="cells per axis (default: workload size)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="fp64, or mixed: float contractions with float64 state, limiters and dt")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration)")
    ap.add_argument("--summarize-profile", metavar="DIR",
                    help="write the rocprofv3 summary of DIR/{stats,fetch,write,copy_fetch,copy_write}")
    ap.add_argument("--profile-command", default="", help="command text recorded in the summary")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.summarize_profile:
        from paper_2509_04673_amd import workloads
        kw = {} if args.n is None else dict(n=args.n)
        if args.workload == "euler_batch":
            name = f"euler_batch_{args.count}_q2_{args.precision}_stage_kernels.md"
        else:
            name = profile_name(workloads.make(args.workload, seed=0, **kw), args.precision)
        summarize_profile(args.summarize_profile, os.path.join(PROFILE_DIR, name),
                          args.profile_command, COPY_PROBE_BYTES)
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "decomposition is described, not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2509_04673_amd import cem, workloads

    if args.workload == "euler_batch":
        return bench_batch(args)

    kw = {} if args.n is None else dict(n=args.n)
    wl = workloads.make(args.workload, seed=0, **kw)
    print(f"[bench] workload {wl.name} d={wl.d} p={wl.p} n={wl.n} dofs={wl.dofs} "
          f"precision={args.precision}", flush=True)
    dev = torch.device("cuda:0")
    s = cem.Solver.from_workload(wl, device="cuda:0", precision=args.precision)
    s.upload(wl.u0)
    if wl.kind != "euler":
        s.set_bounds()
    dt, cfl = (wl.dt, 0.0) if wl.dt > 0 else (0.0, wl.cfl)

    # warm-up with every kernel timed (direct launches): the dominant kernel
    # (at least one step, also with --warmup 0, to find that kernel)
    nwarm = max(1, args.warmup)
    cem.cem_set_timing(s.ctx, (1 << len(cem.KERNELS)) - 1)
    for _ in range(nwarm):
        s.step(dt, cfl)
    warm = cem.cem_kernel_times(s.ctx)
    # the dominant kernel among the ids that are one device launch per stage
    # (the line-operator ids cover one launch per axis)
    single = {k: v for k, v in warm.items() if v[1] == 3 * nwarm}
    dominant = max(single, key=lambda k: single[k][0])
    print("[bench] warm-up kernel ms: " + ", ".join(f"{k}={v[0]:.2f}/{v[1]}" for k, v in warm.items()
                                                   if v[1]), flush=True)

    # timed region: whole steps replayed as HIP graphs, no events inside
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

    # roofline pass right after, same steps launched directly with HIP events
    # on the library's stream around every launch of the dominant kernel
    nroof = min(args.steps, 50)
    cem.cem_set_timing(s.ctx, 1 << cem.KERNELS.index(dominant))
    for _ in range(nroof):
        s.step(dt, cfl)
    kt = cem.cem_kernel_times(s.ctx)
    cem.cem_set_timing(s.ctx, 0)
    s.close()

    stages = 3 * args.steps
    value = wl.dofs * stages / (ms * 1e-3)
    mixed = args.precision == "mixed"
    nbytes, nflops = kernel_work(dominant, wl, s.N, s.E, s.m, mixed)
    if dominant == "grad_line":
        # one launch may carry the passes of several axes
        per_stage = warm[dominant][1] / (3 * nwarm)
        nbytes, nflops = nbytes * wl.d / per_stage, nflops * wl.d / per_stage
    kms, kcnt = kt[dominant]
    avg_s = (kms / kcnt) * 1e-3 if kcnt else float("nan")
    # the bound is the larger of the two algorithmic lower bounds
    fpeak = FP32_VECTOR_TFLOPS if mixed else FP64_VECTOR_TFLOPS
    if nbytes / (HBM_PEAK_GBS * 1e9) >= nflops / (fpeak * 1e12):
        bound, achieved, peak, unit = "hbm", nbytes / avg_s / 1e9, HBM_PEAK_GBS, "GB/s"
    else:
        bound, achieved, peak, unit = "alu", nflops / avg_s / 1e12, fpeak, "TFLOP/s"
    traffic, prof = profiled_traffic(wl, DEVICE_KERNELS[dominant], args.precision)
    roof = dict(bound=bound, kernel=dominant, achieved=achieved, peak=peak, unit=unit,
                frac=achieved / peak, traffic=traffic, algorithmic_bytes=nbytes, algorithmic_flops=nflops,
                avg_launch_us=avg_s * 1e6, launches=kcnt,
                profiled_avg_us=None if prof is None or traffic is None else
                next(r["avg_us"] for n, r in prof["kernels"].items()
                     if any(k in n for k in DEVICE_KERNELS[dominant])))

    cpu = None
    if not args.no_cpu_baseline:
        print(f"[bench] timing the oracle for ~{args.cpu_seconds:.0f} s", flush=True)
        cpu = cpu_baseline(wl, args.cpu_seconds)

    out = dict(metric="DOF*RK-stage updates/s", value=value, unit="DOF*stage/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=ms / args.steps,
               higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f64" if args.precision == "fp64" else "f32+f64",
               data="synthetic",
               config=dict(workload=wl.name, dim=wl.d, degree=wl.p, cells=list(wl.n),
                           dofs=wl.dofs, physics=wl.kind, dt=wl.dt if wl.dt > 0 else None,
                           cfl=None if wl.dt > 0 else wl.cfl, seed=0,
                           wall_s=wall, violations=chk["violations"],
                           clamped=chk["clamped"]),
               roofline=roof, cpu_baseline=cpu)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
