"""Build libpssgp.so (HIP for gfx950) in-tree.

The kernels are templated on the state layout; each layout's filter,
smoother and adjoint kernels are compiled in their own translation unit so
that the compilation runs in parallel. ``python -m paper_2102_09964_amd.build``
builds; the library lands next to this file.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpssgp.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# packed FP32 instructions are disabled for all device code (v_pk_* forms
# are avoided on this target); the host pass warns about the unknown
# feature, which is harmless.
# Register spills go to scratch memory, not to accumulation registers: with
# spills to accumulation registers the FP64 adjoint fold at d = 8 (512
# registers per lane) returned wrong chunk maps in one build of otherwise
# unchanged source, deterministically, and correct ones with this option
# (the kernels that reach the register limit in FP32 allocate accumulation
# registers directly and are unaffected).
CFLAGS = ["-O3", "--offload-arch=" + ARCH, "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-mllvm", "-amdgpu-spill-vgpr-to-agpr=0",
          ] + (["-DPSSGP_WITH_GRAD"] if os.path.exists(os.path.join(CSRC, "inst_grad.hip")) else [])

INST_UNITS = ["inst_filter.hip", "inst_smoother.hip", "inst_grad.hip", "inst_plain.hip"]
PLAIN_UNITS = ["model.cpp", "capi.cpp", "dispatch.hip", "batched.hip", "merge.hip", "noalloc.hip",
               "qp_host.cpp", "qp.hip", "plan.cpp"]


def layouts():
    """(B0, B1) pairs from the PSSGP_LAYOUTS list in launch.h."""
    src = open(os.path.join(CSRC, "launch.h")).read()
    m = re.search(r"#define PSSGP_LAYOUTS\(X\)(.*)", src)
    return [(int(a), int(b)) for a, b in re.findall(r"X\((\d+),\s*(\d+)\)", m.group(1))]


def _compile(src, obj, extra):
    cmd = [HIPCC] + CFLAGS + extra + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(jobs: int | None = None, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    tasks = []
    for u in PLAIN_UNITS:
        src = os.path.join(CSRC, u)
        if os.path.exists(src):
            tasks.append((src, os.path.join(BUILD, u + ".o"), []))
    for u in INST_UNITS:
        src = os.path.join(CSRC, u)
        if not os.path.exists(src):
            continue
        for b0, b1 in layouts():
            obj = os.path.join(BUILD, "%s.%d_%d.o" % (u, b0, b1))
            tasks.append((src, obj, ["-DINST_B0=%d" % b0, "-DINST_B1=%d" % b1]))
    jobs = jobs or min(len(tasks), max(1, min(16, os.cpu_count() or 1)))
    if verbose:
        print("building %d units with %d jobs" % (len(tasks), jobs), flush=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda a: _compile(*a), tasks))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB, flush=True)
    return LIB


if __name__ == "__main__":
    build(int(sys.argv[1]) if len(sys.argv) > 1 else None)
