"""Build libcem.so (HIP, gfx950) in-tree.

Usage: python -m paper_2509_04673_amd.build [--jobs N]
The host-only table code is compiled with g++, the HIP translation unit with
hipcc for gfx950; packed FP32 instructions are disabled for all device code.
"""
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libcem.so")
BUILD = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("CEM_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics", "-ffp-contract=fast"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    t0 = time.time()
    tables_o = os.path.join(BUILD, "tables.o")
    api_o = os.path.join(BUILD, "api.o")
    procs = [
        subprocess.Popen(["g++", "-O2", "-std=c++17", "-fPIC", "-c",
                          os.path.join(CSRC, "tables.cpp"), "-o", tables_o]),
        subprocess.Popen([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, "api.hip"), "-o", api_o]),
    ]
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("compilation failed")
    tmp = OUT + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", api_o, tables_o, "-o", tmp])
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT} in {time.time() - t0:.1f}s", flush=True)
    return OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
