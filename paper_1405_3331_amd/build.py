"""Build the HIP library ``libcuesim.so`` for gfx950 in-tree.

hipcc compiles every ``csrc/*.hip`` translation unit for the MI355X (gfx950) with packed
FP32 instructions disabled, no fast-math and no floating-point contraction: every fused
multiply-add is an explicit ``fmaf`` in the source, so an expression rounds the same way in
every kernel it is inlined into and the per-step, tiled and batched paths agree bit for
bit.  The system C++ compiler builds the host-only ``csrc/*.cpp`` ones (parameter
validation), and hipcc links them into one shared library next to this file.
"""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBRARY = os.path.join(HERE, "libcuesim.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=off",
    "-I", INCLUDE, "-I", CSRC,
]


HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-I", INCLUDE, "-I", CSRC]


def sources():
    """HIP translation units (device and host code) and plain host C++ ones."""
    return (sorted(glob.glob(os.path.join(CSRC, "*.hip"))) +
            sorted(glob.glob(os.path.join(CSRC, "*.cpp"))))


def build(verbose=False, jobs=8):
    """Compile every translation unit (in parallel) and link ``libcuesim.so``."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(ROOT, "_build", "obj")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        if src.endswith(".cpp"):   # host-only code: the system C++ compiler
            cmd = [os.environ.get("CXX", "g++"), *HOST_FLAGS, "-c", src, "-o", obj]
        else:
            cmd = [hipcc, *HIPCC_FLAGS, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    tmp = LIBRARY + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIBRARY)
    return LIBRARY


def _wait(item):
    src, proc = item
    _, err = proc.communicate()
    lines = [l for l in err.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if proc.returncode != 0:
        sys.stderr.write(err)
        raise RuntimeError(f"hipcc failed on {src}")
    if lines:
        sys.stderr.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
