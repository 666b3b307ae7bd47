"""The C-ABI library loads on the host and exports every symbol that
include/cem.h declares; host-side argument validation (no GPU work)."""
import ctypes
import os
import re

import pytest

from paper_2509_04673_amd import cem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cem.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cem_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("cem_create", "cem_bind", "cem_rk_stage", "cem_step", "cem_check_invariants",
                 "cem_upload_state", "cem_download_state", "cem_debug_tap", "cem_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = cem.lib()
    for name in _declared():
        assert hasattr(lib, name), name
    bound = {s[0] for s in cem._SIGS}
    assert set(_declared()) == bound


def _desc(d=2, p=2, n=(8, 8), kind=cem.KPP, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    mesh = cem.MeshDesc(d, p, (ctypes.c_int * 3)(*(list(n) + [1] * (3 - len(n)))),
                        (ctypes.c_double * 3)(*lo), (ctypes.c_double * 3)(*hi))
    phys = cem.PhysicsDesc(kind, (ctypes.c_double * 3)(1.0, 0.0, 0.0), 1.4)
    return mesh, phys


def test_create_and_sizes_on_host():
    mesh, phys = _desc()
    ctx = cem.cem_create(mesh, phys, cem.cem_params_default(), 0)
    try:
        N, E, m = cem.cem_sizes(ctx)
        assert (N, E, m) == (16 * 16, 64, 1)
        assert cem.cem_workspace_bytes(ctx) > 8 * N * 4
        assert cem.cem_tap_size(ctx, cem.TAPS["elemvec"]) == 9 * 64
    finally:
        cem.cem_destroy(ctx)


@pytest.mark.parametrize("bad", ["dim", "degree", "cells", "aspect", "gamma", "velocity", "precision",
                                 "flux_mode", "bounds", "contrib", "q1_degree", "too_large"])
def test_create_rejects_invalid_configurations(bad):
    kw = dict()
    mesh, phys = _desc()
    prm = cem.cem_params_default()
    if bad == "precision":
        prm.precision = 5
    elif bad == "flux_mode":
        prm.flux_mode = 3
    elif bad == "bounds":
        prm.bounds = 2
    elif bad == "contrib":
        prm.contrib = 2
    elif bad == "q1_degree":
        prm.contrib = cem.CONTRIB_Q1     # the default mesh has degree 2
    elif bad == "too_large":
        # m N must stay below 2^31 (32-bit device index arithmetic)
        mesh.dim, mesh.degree = 3, 2
        for k in range(3):
            mesh.n[k] = 700
            mesh.hi[k] = 1.0
        phys.kind = cem.EULER
        phys.gamma_gas = 1.4
    elif bad == "dim":
        mesh.dim = 4
    elif bad == "degree":
        mesh.degree = 7
    elif bad == "cells":
        mesh.n[0] = 1
    elif bad == "aspect":
        mesh.hi[1] = 2.0
    elif bad == "gamma":
        phys.kind = cem.EULER
        phys.gamma_gas = 2.0
    elif bad == "velocity":
        phys.kind = cem.ADVECTION
        phys.velocity[0] = 0.0
    with pytest.raises(cem.CemError) as ei:
        cem.cem_create(mesh, phys, prm, 0)
    assert ei.value.status == -1
    del kw


def test_calls_before_bind_are_rejected():
    mesh, phys = _desc()
    ctx = cem.cem_create(mesh, phys, cem.cem_params_default(), 0)
    try:
        with pytest.raises(cem.CemError):
            cem.cem_rk_stage(ctx, 0, 1e-3)
        with pytest.raises(cem.CemError):
            cem.cem_check_invariants(ctx)
    finally:
        cem.cem_destroy(ctx)


def test_line_kernel_mode_is_validated_on_the_host():
    mesh, phys = _desc()
    ctx = cem.cem_create(mesh, phys, cem.cem_params_default(), 0)
    try:
        for mode in (0, 1, 2):
            cem.cem_set_line_kernels(ctx, mode)
        for bad in (-1, 3):
            with pytest.raises(cem.CemError):
                cem.cem_set_line_kernels(ctx, bad)
    finally:
        cem.cem_destroy(ctx)


def _line_desc(p=2, n=10, kind=cem.EULER, bc=("state", "outflow"), state=(1.0, 0.2, 2.5)):
    mesh, phys = _desc(d=1, p=p, n=(n,), kind=kind)
    for s, k in enumerate(bc):
        mesh.bc[s] = cem.BCS[k]
        for q, v in enumerate(state):
            mesh.bc_state[s][q] = v
    return mesh, phys


def test_line_create_and_sizes_on_host():
    # a non-periodic line holds p n + 1 nodes
    for p, n in ((1, 7), (2, 10), (3, 200)):
        mesh, phys = _line_desc(p, n)
        ctx = cem.cem_create(mesh, phys, cem.cem_params_default(), 0)
        try:
            assert cem.cem_sizes(ctx) == (p * n + 1, n, 3)
        finally:
            cem.cem_destroy(ctx)


@pytest.mark.parametrize("bad", ["one_periodic", "two_d", "mixed", "subcell", "q1", "wall_scalar",
                                 "state_pressure", "state_nan", "scalar_outside", "kind"])
def test_line_create_rejects_invalid_boundaries(bad):
    mesh, phys = _line_desc()
    prm = cem.cem_params_default()
    if bad == "one_periodic":
        mesh.bc[1] = cem.BC_PERIODIC
    elif bad == "two_d":
        mesh.dim, mesh.n[1], mesh.hi[1] = 2, 10, 1.0
    elif bad == "mixed":
        prm.precision = cem.FP32_MIXED
    elif bad == "subcell":
        prm.flux_mode = cem.FLUX_SUBCELL
    elif bad == "q1":
        mesh, phys = _line_desc(p=1, kind=cem.ADVECTION, bc=("outflow", "outflow"))
        prm.contrib = cem.CONTRIB_Q1
    elif bad == "wall_scalar":
        mesh, phys = _line_desc(kind=cem.ADVECTION, bc=("wall", "outflow"))
    elif bad == "state_pressure":
        mesh.bc_state[0][2] = 0.01          # E below the kinetic energy
    elif bad == "state_nan":
        mesh.bc_state[0][0] = float("nan")
    elif bad == "scalar_outside":
        mesh, phys = _line_desc(kind=cem.ADVECTION, bc=("state", "outflow"), state=(3.0,))
        prm.u_min, prm.u_max = 0.0, 1.0
    elif bad == "kind":
        mesh.bc[0] = 7
    with pytest.raises(cem.CemError) as ei:
        cem.cem_create(mesh, phys, prm, 0)
    assert ei.value.status == -1


def test_batch_refuses_boundaries():
    # (a 2D Euler batch, which the batched form supports, with boundary
    # conditions set on its mesh)
    mesh, phys = _desc(kind=cem.EULER)
    mesh.bc[0] = mesh.bc[1] = cem.BC_OUTFLOW
    with pytest.raises(cem.CemError) as ei:
        cem.cem_batch_create([mesh], phys, cem.cem_params_default(), 0)
    assert "periodic" in str(ei.value)


def test_nonconvex_flux_is_one_dimensional():
    mesh, phys = _desc(d=1, p=2, n=(12,), kind=cem.NONCONVEX)
    ctx = cem.cem_create(mesh, phys, cem.cem_params_default(), 0)
    cem.cem_destroy(ctx)
    mesh, phys = _line_desc(kind=cem.NONCONVEX, bc=("state", "outflow"), state=(0.0,))
    ctx = cem.cem_create(mesh, phys, cem.cem_params_default(), 0)
    cem.cem_destroy(ctx)
    mesh, phys = _desc(d=2, kind=cem.NONCONVEX)
    with pytest.raises(cem.CemError):
        cem.cem_create(mesh, phys, cem.cem_params_default(), 0)
