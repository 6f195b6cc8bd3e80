"""Build libpbit.so (HIP kernels for gfx950 + host runtime) in-tree.

    python -m paper_2007_07379_amd.build

Every source is rebuilt on each call.  HIP sources are compiled with
hipcc --offload-arch=gfx950; packed FP32 instructions are disabled for all
device code.  The circuit compiler is host-only C++ built with
-ffp-contract=off so its FP64 threshold arithmetic is the written sequence.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "libpbit.so")
BUILD = os.path.join(ROOT, "_build")

ARCH = "gfx950"
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]

SOURCES = [
    # (file, compiler)
    ("compile.cpp", "host"),
    ("abi.cpp", "hip-host"),
    ("runtime.cpp", "hip-host"),
    ("tune.cpp", "hip-host"),
    ("jit.cpp", "hip-host"),
    ("proposal.cpp", "hip"),
    ("blaslt.cpp", "hip-host"),
    ("autotune.cpp", "hip-host"),
    ("gibbs.hip", "hip"),
    ("gibbs_pair.hip", "hip"),
    ("made.hip", "hip"),
    ("mh.hip", "hip"),
    ("batched.hip", "hip"),
    ("keyhist.hip", "hip"),
    ("shor.hip", "hip"),
]


def _cmd(src, kind, obj):
    path = os.path.join(CSRC, src)
    if kind == "host":
        return ["g++", "-ffp-contract=off", "-Wall", "-Wno-unused-function"] + COMMON + ["-c", path, "-o", obj]
    if kind == "hip-host":
        return [HIPCC, "--offload-arch=" + ARCH] + COMMON + DEVICE_FLAGS + ["-c", path, "-o", obj]
    return [HIPCC, "--offload-arch=" + ARCH] + COMMON + DEVICE_FLAGS + ["-c", path, "-o", obj]


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for src, kind in SOURCES:
        if not os.path.exists(os.path.join(CSRC, src)):
            continue
        obj = os.path.join(BUILD, src + ".o")
        jobs.append((src, _cmd(src, kind, obj), obj))

    def run(job):
        src, cmd, obj = job
        r = subprocess.run(cmd, capture_output=True, text=True)
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
        if r.returncode != 0:
            raise RuntimeError("build of %s failed:\n%s\n%s" % (src, " ".join(cmd), msg))
        if verbose and msg.strip():
            print(msg)
        return obj

    workers = min(len(jobs), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(workers) as ex:
        objs = list(ex.map(run, jobs))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lhiprtc", "-lhipblaslt"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stdout + r.stderr))
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
