"""Build the gfx950 shared library ``libscomp.so`` in-tree.

Every source under ``csrc/`` is compiled by hipcc for gfx950 (the kernel
instantiations of ``dispatch.hip`` once per part, in parallel) and linked
into ``paper_2205_03354_amd/libscomp.so``. Object files go to ``_build/``.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libscomp.so")
ARCH = "gfx950"
NPARTS = 13

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

# Packed FP32 instructions are disabled (the compiler would otherwise form
# v_pk_* FP32 ops from float2/float4 code).
BASE_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "-Wno-unused-variable", "-Wno-unused-but-set-variable",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(HERE, "..", "include"),
]


def _jobs():
    n = os.cpu_count() or 4
    env = os.environ.get("MAX_JOBS")
    if env and env.isdigit():
        n = int(env)
    return max(1, min(n, 16))


def _units():
    units = []
    for name in ("abi.cpp", "stencil.cpp", "solver.cpp", "server.cpp", "precond.cpp", "imex.cpp"):
        units.append((os.path.join(CSRC, name), os.path.join(BUILD, name + ".o"), ["-x", "hip"]))
    for name in ("launch_host.hip", "elementwise.hip", "csr.hip", "small.hip", "varcoef.hip"):
        units.append((os.path.join(CSRC, name), os.path.join(BUILD, name + ".o"), []))
    for part in range(NPARTS):
        units.append((os.path.join(CSRC, "dispatch.hip"), os.path.join(BUILD, f"dispatch_{part}.o"),
                      [f"-DSC_PART={part}"]))
    return units


def _compile(unit):
    src, obj, extra = unit
    cmd = [HIPCC] + BASE_FLAGS + extra + ["-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (p.stderr or "").splitlines() if "packed-fp32-ops" not in ln]
    return p.returncode, " ".join(cmd), "\n".join(msgs)


def build(verbose: bool = False) -> str:
    """Compile every HIP source for gfx950 and link libscomp.so (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    units = _units()
    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        results = list(ex.map(_compile, units))
    failed = [r for r in results if r[0] != 0]
    for rc, cmd, msg in results:
        if verbose or rc != 0:
            if msg.strip():
                print(msg, file=sys.stderr)
    if failed:
        raise RuntimeError("hipcc failed:\n" + "\n".join(r[1] for r in failed))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + [u[1] for u in units] + \
        ["-L/opt/rocm/lib", "-lrocblas", "-lrocsparse", "-lrocfft", "-Wl,-rpath,/opt/rocm/lib"]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
