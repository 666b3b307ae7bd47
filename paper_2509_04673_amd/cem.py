"""Thin Python binding of libcem.so (C ABI declared in include/cem.h).

Argument marshalling only: every step of the stage runs in the HIP kernels
of the library.  PyTorch provides the device memory (state arrays and the
workspace) and the stream.  The module fails loudly when the library is
missing; there is no fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libcem.so")

ADVECTION, KPP, EULER, NONCONVEX = 0, 1, 2, 3
KINDS = {"advection": ADVECTION, "kpp": KPP, "euler": EULER, "nonconvex": NONCONVEX}
FP64, FP32_MIXED = 0, 1
PRECISIONS = {"fp64": FP64, "mixed": FP32_MIXED}
FLUX_LIMIT, FLUX_SUBCELL, FLUX_SHRINK = 0, 1, 2
FLUX_MODES = {"limit": FLUX_LIMIT, "subcell": FLUX_SUBCELL, "shrink": FLUX_SHRINK}
BOUNDS_GLOBAL, BOUNDS_LOCAL = 0, 1
BOUNDS = {"global": BOUNDS_GLOBAL, "local": BOUNDS_LOCAL}
CONTRIB_AEC, CONTRIB_Q1 = 0, 1
CONTRIBS = {"aec": CONTRIB_AEC, "q1": CONTRIB_Q1}
BC_PERIODIC, BC_STATE, BC_OUTFLOW, BC_WALL = 0, 1, 2, 3
BCS = {"periodic": BC_PERIODIC, "state": BC_STATE, "outflow": BC_OUTFLOW, "wall": BC_WALL}
STATUS = {0: "CEM_OK", -1: "CEM_EINVAL", -2: "CEM_EHIP", -3: "CEM_ENOMEM",
          -4: "CEM_ECFL", -5: "CEM_EIDP"}
TAPS = dict(g=0, r=1, udot=2, gamma=3, nu=4, dt_e=5, ue=6, ubarL=7, ubar=8, beta=9,
            fA=10, elemvec=11, bounds=12)


class CemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class MeshDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("degree", ctypes.c_int), ("n", ctypes.c_int * 3),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("bc", ctypes.c_int * 2), ("bc_state", (ctypes.c_double * 5) * 2)]


def set_mesh_bc(mesh, bc):
    """bc: None (periodic) or ((kind, state), (kind, state)) for the ends at
    lo[0] and hi[0]; kind a key of BCS, state the conserved values of a
    "state" end (else None)."""
    if bc is None:
        return
    for s, (kind, state) in enumerate(bc):
        mesh.bc[s] = BCS[kind] if isinstance(kind, str) else int(kind)
        if state is not None:
            vals = list(np.asarray(state, dtype=np.float64).ravel())
            for q, v in enumerate(vals[:5]):
                mesh.bc_state[s][q] = float(v)


class PhysicsDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("velocity", ctypes.c_double * 3),
                ("gamma_gas", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("q", ctypes.c_double), ("r", ctypes.c_double), ("eps", ctypes.c_double),
                ("w_lin", ctypes.c_double), ("eps_pos", ctypes.c_double),
                ("clamp_ulps", ctypes.c_double), ("gamma_mode", ctypes.c_int),
                ("alpha_mode", ctypes.c_int), ("beta_mode", ctypes.c_int),
                ("u_min", ctypes.c_double), ("u_max", ctypes.c_double),
                ("precision", ctypes.c_int), ("flux_mode", ctypes.c_int), ("bounds", ctypes.c_int),
                ("contrib", ctypes.c_int)]


class Invariants(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("min_dt_e", ctypes.c_double),
                ("cfl_violated", ctypes.c_int), ("clamped", ctypes.c_longlong),
                ("violations", ctypes.c_longlong), ("m", ctypes.c_int),
                ("u_min", ctypes.c_double * 5), ("u_max", ctypes.c_double * 5),
                ("mass", ctypes.c_double * 5), ("rho_min", ctypes.c_double),
                ("p_min", ctypes.c_double), ("nonfinite", ctypes.c_longlong),
                ("state_violations", ctypes.c_longlong)]


# (name, restype, argtypes) of every exported symbol
_P = ctypes.c_void_p
_SIGS = [
    ("cem_params_default", ctypes.c_int, [ctypes.POINTER(Params)]),
    ("cem_create", ctypes.c_int, [ctypes.POINTER(MeshDesc), ctypes.POINTER(PhysicsDesc),
                                  ctypes.POINTER(Params), _P, ctypes.POINTER(_P)]),
    ("cem_sizes", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_longlong),
                                 ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_int)]),
    ("cem_workspace_bytes", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    ("cem_bind", ctypes.c_int, [_P, _P, _P, _P, ctypes.c_size_t]),
    ("cem_upload_state", ctypes.c_int, [_P, _P]),
    ("cem_download_state", ctypes.c_int, [_P, _P]),
    ("cem_set_bounds", ctypes.c_int, [_P, ctypes.c_int, ctypes.c_double, ctypes.c_double]),
    ("cem_rk_stage", ctypes.c_int, [_P, ctypes.c_int, ctypes.c_double, ctypes.c_double]),
    ("cem_step", ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double]),
    ("cem_check_invariants", ctypes.c_int, [_P, ctypes.POINTER(Invariants)]),
    ("cem_reset_counters", ctypes.c_int, [_P]),
    ("cem_debug_tap", ctypes.c_int, [_P, ctypes.c_int, _P, ctypes.c_size_t]),
    ("cem_tap_size", ctypes.c_size_t, [_P, ctypes.c_int]),
    ("cem_set_graphs", ctypes.c_int, [_P, ctypes.c_int]),
    ("cem_set_line_kernels", ctypes.c_int, [_P, ctypes.c_int]),
    ("cem_set_fused_update", ctypes.c_int, [_P, ctypes.c_int]),
    ("cem_state_modified", ctypes.c_int, [_P]),
    ("cem_set_timing", ctypes.c_int, [_P, ctypes.c_uint]),
    ("cem_kernel_times", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_longlong), ctypes.c_int]),
    ("cem_step_static", ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_int]),
    ("cem_destroy", None, [_P]),
    ("cem_last_error", ctypes.c_char_p, []),
    ("cem_batch_create", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(MeshDesc), ctypes.POINTER(PhysicsDesc),
                                        ctypes.POINTER(Params), _P, ctypes.POINTER(_P)]),
    ("cem_batch_offsets", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_longlong), ctypes.c_int]),
    ("cem_batch_workspace_bytes", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    ("cem_batch_bind", ctypes.c_int, [_P, _P, _P, _P, ctypes.c_size_t]),
    ("cem_batch_upload_state", ctypes.c_int, [_P, _P]),
    ("cem_batch_download_state", ctypes.c_int, [_P, _P]),
    ("cem_batch_set_bounds", ctypes.c_int, [_P, ctypes.c_int, ctypes.c_double, ctypes.c_double]),
    ("cem_batch_step", ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double, ctypes.c_int]),
    ("cem_batch_set_graphs", ctypes.c_int, [_P, ctypes.c_int]),
    ("cem_batch_reset_counters", ctypes.c_int, [_P]),
    ("cem_batch_check_invariants", ctypes.c_int, [_P, ctypes.POINTER(Invariants), ctypes.c_int]),
    ("cem_batch_set_plan", ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    ("cem_batch_set_line_kernels", ctypes.c_int, [_P, ctypes.c_int]),
    ("cem_batch_set_fused_update", ctypes.c_int, [_P, ctypes.c_int]),
    ("cem_batch_set_timing", ctypes.c_int, [_P, ctypes.c_uint]),
    ("cem_batch_kernel_times", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_longlong), ctypes.c_int]),
    ("cem_batch_autotune", ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double, ctypes.c_int, _P,
                                          ctypes.c_size_t, ctypes.c_char_p, ctypes.c_size_t]),
    ("cem_batch_destroy", None, [_P]),
]

_lib = None


def lib():
    """Load libcem.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is missing: build it with "
                               "`python -m paper_2509_04673_amd.build`")
        handle = ctypes.CDLL(LIBPATH)
        for name, res, args in _SIGS:
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def _check(status):
    if status != 0:
        raise CemError(status, lib().cem_last_error().decode())
    return status


# -- one Python function per C entry point ---------------------------------
def cem_params_default():
    p = Params()
    _check(lib().cem_params_default(ctypes.byref(p)))
    return p


def make_params(params):
    """cem_params from the defaults and keyword overrides; precision,
    flux_mode, bounds and contrib also take their names ("fp64" / "mixed",
    "limit" / "subcell" / "shrink", "global" / "local", "aec" / "q1")."""
    prm = cem_params_default()
    for k, v in params.items():
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        if k == "flux_mode" and isinstance(v, str):
            v = FLUX_MODES[v]
        if k == "bounds" and isinstance(v, str):
            v = BOUNDS[v]
        if k == "contrib" and isinstance(v, str):
            v = CONTRIBS[v]
        setattr(prm, k, v)
    return prm


def cem_create(mesh, phys, prm, stream):
    ctx = _P()
    _check(lib().cem_create(ctypes.byref(mesh), ctypes.byref(phys), ctypes.byref(prm),
                            _P(stream), ctypes.byref(ctx)))
    return ctx


def cem_sizes(ctx):
    N, E, m = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_int()
    _check(lib().cem_sizes(ctx, ctypes.byref(N), ctypes.byref(E), ctypes.byref(m)))
    return N.value, E.value, m.value


def cem_workspace_bytes(ctx):
    b = ctypes.c_size_t()
    _check(lib().cem_workspace_bytes(ctx, ctypes.byref(b)))
    return b.value


def cem_bind(ctx, u_ptr, u_base_ptr, ws_ptr, ws_bytes):
    _check(lib().cem_bind(ctx, _P(u_ptr), _P(u_base_ptr), _P(ws_ptr), ws_bytes))


def cem_upload_state(ctx, host):
    host = np.ascontiguousarray(host, dtype=np.float64)
    _check(lib().cem_upload_state(ctx, host.ctypes.data))


def cem_download_state(ctx, out):
    assert out.dtype == np.float64 and out.flags.c_contiguous
    _check(lib().cem_download_state(ctx, out.ctypes.data))
    return out


def cem_set_bounds(ctx, from_state, u_min=0.0, u_max=0.0):
    _check(lib().cem_set_bounds(ctx, int(from_state), float(u_min), float(u_max)))


def cem_rk_stage(ctx, stage, dt, cfl=0.0):
    _check(lib().cem_rk_stage(ctx, int(stage), float(dt), float(cfl)))


def cem_step(ctx, dt, cfl=0.0):
    _check(lib().cem_step(ctx, float(dt), float(cfl)))


def cem_check_invariants(ctx, raise_on_failure=True):
    inv = Invariants()
    st = lib().cem_check_invariants(ctx, ctypes.byref(inv))
    if raise_on_failure:
        _check(st)
    return inv, st


def cem_reset_counters(ctx):
    _check(lib().cem_reset_counters(ctx))


def cem_tap_size(ctx, tap):
    return int(lib().cem_tap_size(ctx, int(tap)))


def cem_debug_tap(ctx, tap, dst_ptr, count):
    _check(lib().cem_debug_tap(ctx, int(tap), _P(dst_ptr), int(count)))


KERNELS = ["grad_line", "elem1", "stage_dt", "gather_r", "mass_line", "elem2", "update", "elem1r"]


def cem_set_graphs(ctx, enable):
    _check(lib().cem_set_graphs(ctx, int(bool(enable))))


def cem_set_line_kernels(ctx, mode):
    _check(lib().cem_set_line_kernels(ctx, int(mode)))


def cem_set_fused_update(ctx, enable):
    _check(lib().cem_set_fused_update(ctx, int(bool(enable))))


def cem_state_modified(ctx):
    _check(lib().cem_state_modified(ctx))


def cem_set_timing(ctx, mask):
    _check(lib().cem_set_timing(ctx, int(mask)))


def cem_kernel_times(ctx):
    n = len(KERNELS)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_longlong * n)()
    _check(lib().cem_kernel_times(ctx, ms, cnt, n))
    return {KERNELS[i]: (ms[i], cnt[i]) for i in range(n)}


def cem_step_static(ctx, u_ptr, u_base_ptr, dt=0.0, cfl=0.0, nsteps=1):
    _check(lib().cem_step_static(ctx, _P(u_ptr), _P(u_base_ptr), float(dt), float(cfl), int(nsteps)))


STATIC_WORKSPACE_BYTES = 64 << 20     # CEM_STATIC_WORKSPACE_BYTES of include/cem.h


def cem_destroy(ctx):
    lib().cem_destroy(ctx)


# -- convenience wrapper owning the torch buffers ---------------------------
class Solver:
    """A bound context: state u, step base u_base and workspace are torch
    tensors on `device`; all work goes to the current torch stream."""

    def __init__(self, d, p, n, lo, hi, kind, velocity=(1.0, 0.0, 0.0), gamma_gas=1.4,
                 device="cuda:0", bc=None, **params):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        mesh = MeshDesc(d, p, (ctypes.c_int * 3)(*(list(n) + [1] * (3 - d))),
                        (ctypes.c_double * 3)(*(list(lo) + [0.0] * (3 - d))),
                        (ctypes.c_double * 3)(*(list(hi) + [1.0] * (3 - d))))
        set_mesh_bc(mesh, bc)
        phys = PhysicsDesc(KINDS[kind], (ctypes.c_double * 3)(*(list(velocity) + [0.0] * 3)[:3]),
                           gamma_gas)
        prm = make_params(params)
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = cem_create(mesh, phys, prm, self.stream.cuda_stream)
        self.N, self.E, self.m = cem_sizes(self.ctx)
        self.d, self.p, self.kind = d, p, kind
        nbytes = cem_workspace_bytes(self.ctx)
        self.u = torch.zeros((self.m, self.N), dtype=torch.float64, device=self.device)
        self.u_base = torch.zeros_like(self.u)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        aligned = (base + 255) & ~255
        cem_bind(self.ctx, self.u.data_ptr(), self.u_base.data_ptr(), aligned, nbytes)

    @classmethod
    def from_workload(cls, wl, device="cuda:0", **params):
        params.setdefault("w_lin", wl.w_lin)
        params.setdefault("q", wl.q)
        return cls(wl.d, wl.p, wl.n, wl.lo, wl.hi, wl.kind, wl.velocity, wl.gamma_gas,
                   device=device, bc=getattr(wl, "bc", None), **params)

    def upload(self, host_u):
        cem_upload_state(self.ctx, np.asarray(host_u, dtype=np.float64).reshape(self.m, self.N))

    def download(self):
        out = np.empty((self.m, self.N), dtype=np.float64)
        return cem_download_state(self.ctx, out)

    def set_bounds(self, u_min=None, u_max=None):
        if u_min is None:
            cem_set_bounds(self.ctx, 1)
        else:
            cem_set_bounds(self.ctx, 0, u_min, u_max)

    def stage(self, s, dt=0.0, cfl=0.0):
        cem_rk_stage(self.ctx, s, dt, cfl)

    def step(self, dt=0.0, cfl=0.0):
        cem_step(self.ctx, dt, cfl)

    def set_line_kernels(self, mode):
        """0 vector, 1 matrix cores, 2 by size (see cem_set_line_kernels)."""
        cem_set_line_kernels(self.ctx, mode)

    def set_fused_update(self, enable):
        cem_set_fused_update(self.ctx, enable)

    def set_graphs(self, enable):
        cem_set_graphs(self.ctx, enable)

    def reset_counters(self):
        cem_reset_counters(self.ctx)

    def check(self, raise_on_failure=False):
        inv, st = cem_check_invariants(self.ctx, raise_on_failure)
        m = inv.m
        return dict(status=st, dt=inv.dt, min_dt_e=inv.min_dt_e, cfl_violated=inv.cfl_violated,
                    clamped=inv.clamped, violations=inv.violations,
                    u_min=list(inv.u_min)[:m], u_max=list(inv.u_max)[:m],
                    mass=list(inv.mass)[:m], rho_min=inv.rho_min, p_min=inv.p_min,
                    nonfinite=inv.nonfinite, state_violations=inv.state_violations)

    def tap(self, name):
        tid = TAPS[name]
        n = cem_tap_size(self.ctx, tid)
        buf = self.torch.empty(n, dtype=self.torch.float64, device=self.device)
        cem_debug_tap(self.ctx, tid, buf.data_ptr(), n)
        self.torch.cuda.synchronize(self.device)
        return buf.cpu().numpy()

    def close(self):
        if self.ctx:
            cem_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# -- batched form --------------------------------------------------------------
def cem_batch_create(meshes, phys, prm, stream):
    arr = (MeshDesc * len(meshes))(*meshes)
    b = _P()
    _check(lib().cem_batch_create(len(meshes), arr, ctypes.byref(phys), ctypes.byref(prm), _P(stream),
                                  ctypes.byref(b)))
    return b


def cem_batch_offsets(b, count):
    off = (ctypes.c_longlong * (count + 1))()
    _check(lib().cem_batch_offsets(b, off, count + 1))
    return np.array(off[:], dtype=np.int64)


def cem_batch_workspace_bytes(b):
    n = ctypes.c_size_t()
    _check(lib().cem_batch_workspace_bytes(b, ctypes.byref(n)))
    return n.value


def cem_batch_bind(b, u_ptr, u0_ptr, ws_ptr, nbytes):
    _check(lib().cem_batch_bind(b, _P(u_ptr), _P(u0_ptr), _P(ws_ptr), nbytes))


def cem_batch_upload_state(b, host):
    host = np.ascontiguousarray(host, dtype=np.float64)
    _check(lib().cem_batch_upload_state(b, host.ctypes.data_as(_P)))


def cem_batch_download_state(b, n):
    out = np.empty(n, dtype=np.float64)
    _check(lib().cem_batch_download_state(b, out.ctypes.data_as(_P)))
    return out


def cem_batch_set_bounds(b, from_state, u_min=0.0, u_max=0.0):
    _check(lib().cem_batch_set_bounds(b, int(from_state), float(u_min), float(u_max)))


def cem_batch_step(b, dt, cfl, nsteps):
    _check(lib().cem_batch_step(b, float(dt), float(cfl), int(nsteps)))


def cem_batch_set_graphs(b, enable):
    _check(lib().cem_batch_set_graphs(b, int(bool(enable))))


def cem_batch_reset_counters(b):
    _check(lib().cem_batch_reset_counters(b))


def cem_batch_check_invariants(b, count):
    inv = (Invariants * count)()
    st = lib().cem_batch_check_invariants(b, inv, count)
    return list(inv), st


def cem_batch_set_plan(b, order=0, xlines_cap=2048, ytile_lds_bytes=40960, elem1_kernel=0):
    _check(lib().cem_batch_set_plan(b, int(order), int(xlines_cap), int(ytile_lds_bytes), int(elem1_kernel)))


def cem_batch_set_line_kernels(b, matrix):
    _check(lib().cem_batch_set_line_kernels(b, int(matrix)))


def cem_batch_set_fused_update(b, enable):
    _check(lib().cem_batch_set_fused_update(b, int(bool(enable))))


def cem_batch_set_timing(b, mask):
    _check(lib().cem_batch_set_timing(b, int(mask)))


def cem_batch_kernel_times(b):
    n = len(KERNELS)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_longlong * n)()
    _check(lib().cem_batch_kernel_times(b, ms, cnt, n))
    return {KERNELS[i]: (ms[i], cnt[i]) for i in range(n)}


def cem_batch_autotune(b, dt, cfl, steps, scratch_ptr, scratch_bytes):
    buf = ctypes.create_string_buffer(8192)
    _check(lib().cem_batch_autotune(b, float(dt), float(cfl), int(steps), _P(scratch_ptr), int(scratch_bytes),
                                    buf, len(buf)))
    return buf.value.decode()


def cem_batch_destroy(b):
    lib().cem_batch_destroy(b)


class BatchSolver:
    """Independent problems advanced by the batched kernels: the states are
    one concatenated torch tensor (problem k at offsets[k]:offsets[k+1])."""

    def __init__(self, problems, kind, velocity=(1.0, 0.0, 0.0), gamma_gas=1.4, device="cuda:0", **params):
        """problems: list of (d, p, n, lo, hi) or (d, p, n, lo, hi, bc), bc
        the boundary conditions of a 1D line (see set_mesh_bc)."""
        import torch
        self.torch = torch
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        meshes = []
        for prob in problems:
            d, p, n, lo, hi = prob[:5]
            mesh = MeshDesc(d, p, (ctypes.c_int * 3)(*(list(n) + [1] * (3 - d))),
                            (ctypes.c_double * 3)(*(list(lo) + [0.0] * (3 - d))),
                            (ctypes.c_double * 3)(*(list(hi) + [1.0] * (3 - d))))
            set_mesh_bc(mesh, prob[5] if len(prob) > 5 else None)
            meshes.append(mesh)
        phys = PhysicsDesc(KINDS[kind], (ctypes.c_double * 3)(*(list(velocity) + [0.0] * 3)[:3]), gamma_gas)
        prm = make_params(params)
        self.count = len(problems)
        self.kind = kind
        self.stream = torch.cuda.current_stream(self.device)
        self.b = cem_batch_create(meshes, phys, prm, self.stream.cuda_stream)
        self.offsets = cem_batch_offsets(self.b, self.count)
        nbytes = cem_batch_workspace_bytes(self.b)
        total = int(self.offsets[-1])
        self.u = torch.zeros(total, dtype=torch.float64, device=self.device)
        self.u_base = torch.zeros_like(self.u)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.ws.data_ptr() + 255) & ~255
        cem_batch_bind(self.b, self.u.data_ptr(), self.u_base.data_ptr(), aligned, nbytes)

    def upload(self, states):
        """states: list of per-problem arrays (m, N) or one concatenated array."""
        if isinstance(states, (list, tuple)):
            states = np.concatenate([np.asarray(s, dtype=np.float64).ravel() for s in states])
        cem_batch_upload_state(self.b, states)

    def download(self, split=True):
        flat = cem_batch_download_state(self.b, int(self.offsets[-1]))
        if not split:
            return flat
        return [flat[self.offsets[k]:self.offsets[k + 1]] for k in range(self.count)]

    def set_bounds(self, u_min=None, u_max=None):
        if u_min is None:
            cem_batch_set_bounds(self.b, 1)
        else:
            cem_batch_set_bounds(self.b, 0, u_min, u_max)

    def step(self, dt=0.0, cfl=0.0, nsteps=1):
        cem_batch_step(self.b, dt, cfl, nsteps)

    def autotune(self, dt=0.0, cfl=0.0, steps=2):
        """Pick the fastest plan (see cem_batch_autotune); returns its JSON report."""
        import json
        scratch = self.torch.empty_like(self.u)
        rep = cem_batch_autotune(self.b, dt, cfl, steps, scratch.data_ptr(), scratch.numel() * 8)
        del scratch
        return json.loads(rep)

    def check(self):
        inv, st = cem_batch_check_invariants(self.b, self.count)
        return [dict(status=st, dt=r.dt, min_dt_e=r.min_dt_e, cfl_violated=r.cfl_violated,
                     clamped=r.clamped, violations=r.violations, rho_min=r.rho_min, p_min=r.p_min,
                     mass=list(r.mass)[:r.m], nonfinite=r.nonfinite,
                     state_violations=r.state_violations) for r in inv]

    def close(self):
        if self.b:
            cem_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
