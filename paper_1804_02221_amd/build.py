"""Build the HIP library libesdg.so for gfx950 in place.

One object per polynomial degree (the kernel templates are instantiated for
N = 2..8 in separate translation units that compile in parallel), one object
for the host runtime, linked into ``paper_1804_02221_amd/libesdg.so``.
Objects go to ``_build/`` at the repository root.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libesdg.so")
# the same library with the host code under AddressSanitizer (the kernels are
# not instrumented); loaded by esdg.use_sanitized_build() in a process that
# preloads gcc's ASan runtime (ROCm's clang runtime also intercepts the HSA
# device allocator, which uninstrumented kernels do not need)
LIB_SAN = os.path.join(HERE, "libesdg_hostsan.so")
HOST_SAN = "-Xarch_host -fsanitize=address -Xarch_host -fno-omit-frame-pointer".split()
DEGREES = range(2, 9)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-std=c++17", "-O3", "-fPIC", "--offload-arch=gfx950",
         # packed FP32 instructions off (see DESIGN notes on the toolchain)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", INCLUDE, "-I", CSRC]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
        raise RuntimeError(f"build step failed: {' '.join(cmd)}\n{msg}")
    return r


def build(force: bool = True, jobs: int | None = None, sanitize: bool = False) -> str:
    """Build libesdg.so (or, with sanitize, libesdg_hostsan.so: the host
    code of every object under AddressSanitizer, the same device code)."""
    lib = LIB_SAN if sanitize else LIB
    bdir = os.path.join(BUILD, "hostsan") if sanitize else BUILD
    os.makedirs(bdir, exist_ok=True)
    srcs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp"))]
    newest = max(os.path.getmtime(s) for s in srcs + [os.path.join(INCLUDE, "esdg.h")])
    if not force and os.path.exists(lib) and os.path.getmtime(lib) >= newest:
        return lib
    jobs = jobs or min(8, os.cpu_count() or 4)
    flags = FLAGS + (HOST_SAN if sanitize else [])
    cmds = []
    objs = []
    for n in DEGREES:
        o = os.path.join(bdir, f"esdg_inst_{n}.o")
        cmds.append([HIPCC, *flags, f"-DESDG_N={n}", "-c", os.path.join(CSRC, "esdg_inst.hip"), "-o", o])
        objs.append(o)
    o = os.path.join(bdir, "esdg_runtime.o")
    cmds.append([HIPCC, *flags, "-c", os.path.join(CSRC, "esdg_runtime.hip"), "-o", o])
    objs.append(o)
    with ThreadPoolExecutor(jobs) as ex:
        list(ex.map(_run, cmds))
    tmp = lib + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *(HOST_SAN if sanitize else []), "-o", tmp, *objs])
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(force=True, sanitize="--sanitize" in sys.argv))
