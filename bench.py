"""Benchmark: DOF x RK-stage updates per second of the limited CG-WENO
SSP-RK3 scheme on one MI355X.

Default workload: the 2D KPP problem (flux (sin u, cos u)) on
[-2,2]x[-2.5,1.5] with 256x256 Bernstein Q2 cells (262144 unique DOFs),
float64, fixed dt = 5e-4, seeded disc data.  A step is one full SSP-RK3 step
(three stages, each the whole five-step algorithm: projected gradient, WENO
sensor and residual, consistent-mass solve, facet fluxes with the flux
limiter, element contributions with the slope limiter, assembly and the RK
combination).  Inputs are resident in HBM when the timed region starts.

Prints one JSON line with the throughput, a roofline record of the dominant
kernel (HIP events on the library's stream around the dominant kernel in a pass of
directly launched steps right after the graph-replayed timed region) and the
float64 oracle timed on the host on a bounded sample of the same workload.
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


def kernel_model(name, wl, N, E, m):
    """(bound, algorithmic units per launch, unit) of each kernel.

    Line operators read and write one nodal array: 16 m N bytes.  The gather
    reads the element vectors and writes r; the update reads the element
    vectors, u and u_base and writes u.  The element passes are priced by
    the nodal and per-element arrays they must read and write."""
    d, p = wl.d, wl.p
    nl = (p + 1) ** d
    f8 = 8.0
    if name in ("grad_line", "mass_line"):
        return "hbm", 2 * m * N * f8
    if name == "gather_r":
        return "hbm", (m * nl * E + m * N) * f8
    if name == "update":
        return "hbm", (m * nl * E + 3 * m * N) * f8
    if name == "elem1":
        # reads u, g; writes element residual vectors and per-element data
        return "hbm", ((1 + d) * m * N + m * nl * E + (2 * m + d * m + 3) * E) * f8
    if name == "elem2":
        # reads u, udot, element vectors, per-element data; writes vectors
        return "hbm", (2 * m * N + 2 * m * nl * E + (3 * m + d * m + 1) * E) * f8
    return "hbm", 0.0


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


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="kpp2d", choices=["kpp2d", "adv1d", "euler2d", "euler3d"])
    ap.add_argument("--n", type=int, default=None, help="cells per axis (default: workload size)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design, not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2509_04673_amd import cem, workloads

    kw = {} if args.n is None else dict(n=args.n)
    wl = workloads.make(args.workload, seed=0, **kw)
    print(f"[bench] workload {wl.name} d={wl.d} p={wl.p} n={wl.n} dofs={wl.dofs}", flush=True)
    dev = torch.device("cuda:0")
    s = cem.Solver.from_workload(wl, device="cuda:0")
    s.upload(wl.u0)
    if wl.kind != "euler":
        s.set_bounds()
    dt, cfl = (wl.dt, 0.0) if wl.dt > 0 else (0.0, wl.cfl)

    # warm-up with every kernel timed (direct launches): the dominant kernel
    cem.cem_set_timing(s.ctx, (1 << len(cem.KERNELS)) - 1)
    for _ in range(args.warmup):
        s.step(dt, cfl)
    warm = cem.cem_kernel_times(s.ctx)
    dominant = max(warm, key=lambda k: warm[k][0])
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
    bound, units = kernel_model(dominant, wl, s.N, s.E, s.m)
    kms, kcnt = kt[dominant]
    avg_s = (kms / kcnt) * 1e-3 if kcnt else float("nan")
    if bound == "hbm":
        achieved = units / avg_s / 1e9
        peak, unit = HBM_PEAK_GBS, "GB/s"
    else:
        achieved = units / avg_s / 1e12
        peak, unit = FP64_VECTOR_TFLOPS, "TFLOP/s"
    roof = dict(bound=bound, kernel=dominant, achieved=achieved, peak=peak, unit=unit,
                frac=achieved / peak, traffic=None, avg_launch_us=avg_s * 1e6,
                launches=kcnt)

    cpu = None
    if not args.no_cpu_baseline:
        print(f"[bench] timing the oracle for ~{args.cpu_seconds:.0f} s", flush=True)
        cpu = cpu_baseline(wl, args.cpu_seconds)

    out = dict(metric="DOF*RK-stage updates/s", value=value, unit="DOF*stage/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=ms / args.steps,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64",
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
