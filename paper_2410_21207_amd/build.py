"""Build libseamcarve.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2410_21207_amd.build            # compile if sources changed
    python -m paper_2410_21207_amd.build --force    # always compile

Each source is compiled to an object file in its own hipcc process (in parallel), then the
objects are linked into the shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libseamcarve.so")
SOURCES = [os.path.join(CSRC, n) for n in ("sc_kernels.hip", "sc_object.hip", "sc_forward.hip", "sc_api.cpp")]
HEADERS = [os.path.join(CSRC, "sc_internal.h"), os.path.join(CSRC, "sc_device.h"), os.path.join(ROOT, "include", "sc.h")]
ARCH = os.environ.get("SC_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -packed-fp32-ops: keep the compiler from forming packed fp32 ops (not used here, kept off on gfx950)
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.exists(p) and os.path.getmtime(p) > t for p in SOURCES + HEADERS)


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and not stale():
        return LIB
    tag = "%d" % os.getpid()
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.basename(src) + ".tmp%s.o" % tag)
        cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        objs.append(obj)
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    failed = False
    for p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out)
            failed = True
    tmp = LIB + ".tmp" + tag
    try:
        if failed:
            raise RuntimeError("hipcc failed building libseamcarve.so")
        cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}"] + objs + ["-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed linking libseamcarve.so")
        os.replace(tmp, LIB)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return LIB


if __name__ == "__main__":
    build(force="--force" in sys.argv, verbose=True)
    print(LIB)
