"""Build libbumbar.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbumbar.so")
SOURCES = ["sweep.hip", "sweep_small.hip", "sweep_wide.hip", "sweep_smaj.hip", "sweep32.hip", "sweep_otf.hip", "hessian.hip", "linalg.hip", "covariance.hip", "binning.hip",
           "model.hip", "pmf.hip", "radix.hip", "solver.cpp", "algo.cpp", "server.cpp",
           "sweep_static.cpp", "plan.cpp"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are disabled on purpose (see the design notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wno-unused-result", "-Wshadow",
]


def source_hash() -> str:
    """SHA-256 (first 16 hex digits) of every source file, the public header and
    the compiler flags: bumbar_version() of a library built from this tree ends
    with it, which ties a built libbumbar.so to the sources it came from."""
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp", ".h")))
    for name in files:
        h.update(name.encode() + b"\0")
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(fh.read() + b"\0")
    with open(os.path.join(ROOT, "include", "bumbar.h"), "rb") as fh:
        h.update(fh.read() + b"\0")
    h.update(" ".join(FLAGS[:6]).encode())
    return h.hexdigest()[:16]


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source to an object (in parallel) and link the shared library."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    stamp = f'-DBUMBAR_SOURCE_HASH="{source_hash()}"'
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        cmd = ["hipcc", "-x", "hip", *FLAGS, stamp, "-c", path, "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write(text)
        elif verbose and lines:
            sys.stderr.write("\n".join(lines) + "\n")
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-pthread", "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
