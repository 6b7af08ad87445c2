"""Build libcgh.so (HIP, gfx950) in-tree with hipcc.

Usage: ``python -m paper_2211_09938_amd.build``.  Always recompiles.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcgh.so")
SOURCES = ["dwt.hip", "lut.hip", "reduce.hip", "plan.hip", "ntgemm.hip", "dense.hip", "backward.hip", "exact.hip", "literal.hip", "angular.hip", "peak.hip", "noalloc.hip", "api.cpp", "batch.cpp"]
ARCH = os.environ.get("CGH_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-result",
    "-Wno-unused-const-variable",
]
# Device sources only: keep the compiler from forming packed FP32 VALU
# instructions.  The feature exists only for the GPU target; the host pass of a
# .hip file reports it as unknown and ignores it (the .cpp sources hold no
# device code and do not take it).
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose=False, jobs=4):
    objs = []
    procs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(build_dir, src.replace(".", "_") + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] + DEVICE_FLAGS if src.endswith(".hip") else []
        cmd = [hipcc()] + HIPCC_FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _drain(procs, verbose)
    _drain(procs, verbose)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    _run(cmd, verbose)
    os.replace(tmp, LIB)
    return LIB


def _drain(procs, verbose):
    while procs:
        cmd, p = procs.pop(0)
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + text)
        if verbose and text.strip():
            sys.stderr.write(text)


def _run(cmd, verbose):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + " ".join(cmd) + "\n" + r.stdout.decode(errors="replace"))
    if verbose and r.stdout.strip():
        sys.stderr.write(r.stdout.decode(errors="replace"))


if __name__ == "__main__":
    print(build(verbose=True))
