"""Build the HIP library libgpe.so for gfx950 in-tree (hipcc, no JIT cache).

Usage: python -m paper_1907_01194_amd.build   (or build() from Python).
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgpe.so")
SOURCES = ["lap.hip", "batch_fft.hip", "pointwise.hip", "blas.hip", "mg.hip", "handle.cpp", "solver.cpp", "retract_scalar.cpp",
           "batch.cpp"]
ARCH = os.environ.get("GPE_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are kept out of every kernel.
FLAGS = ["-O3", "-std=c++20", "-fPIC", "--offload-arch=" + ARCH,
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose=False, jobs=None):
    """Compile every source to an object (in parallel) and link libgpe.so."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    cc = hipcc()
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.rsplit(".", 1)[0] + ".o")
        objs.append(obj)
        cmd = [cc] + FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        warn = [l for l in text.splitlines() if "packed-fp32-ops" not in l and "warning: feature flag" not in l]
        if p.returncode != 0:
            failed.append((src, text))
        elif verbose and any(l.strip() for l in warn):
            print(text)
    if failed:
        for src, text in failed:
            sys.stderr.write("---- %s\n%s\n" % (src, text))
        raise RuntimeError("HIP build failed: " + ", ".join(s for s, _ in failed))
    tmp = LIB + ".tmp"
    cmd = [cc, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
