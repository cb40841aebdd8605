"""Build step for the HIP library: compiles csrc/ for gfx950 into
paper_1608_00044_amd/libspchol.so (in-tree, so it travels with the sources)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libspchol.so")
BUILD = os.path.join(ROOT, "_build")
SOURCES = ["symbolic.cpp", "plan.cpp", "schedule.cpp", "api.cpp", "server.cpp", "factor.hip",
           "solve.hip", "refine.hip", "small.hip", "ceiling.hip"]
ARCH = os.environ.get("SPCHOL_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-result",
          "-I" + os.path.join(ROOT, "include")]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-munsafe-fp-atomics"]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        if src.endswith(".hip"):
            cmd = [HIPCC] + COMMON + DEVICE + ["-x", "hip", "-c", path, "-o", obj]
        else:
            cmd = [HIPCC] + COMMON + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                            stderr=subprocess.STDOUT, text=True)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        if out.strip() and (verbose or p.returncode):
            sys.stderr.write(out)
        if p.returncode:
            failed.append(src)
    if failed:
        raise RuntimeError("HIP build failed for: " + ", ".join(failed))
    tmp = LIB + ".tmp%d" % os.getpid()
    # -z defs: an unresolved symbol is a build error, not a load-time one
    cmd = [HIPCC, "-shared", "--offload-arch=" + ARCH, "-Wl,-z,defs", "-pthread", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
