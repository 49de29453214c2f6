"""Build the HIP FDTD library for gfx950 (hipcc, in-tree).

    python paper_2207_06908_amd/csrc/build.py

Produces paper_2207_06908_amd/libmi355fdtd.so (FDTD engine and surrogate network).  Every HIP translation unit
is compiled with FP contraction off (all kernel variants then agree bit for
bit) and with packed FP32 instructions disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
OUT = os.path.join(PKG, "libmi355fdtd.so")
SOURCES = ["fdtd_host.cpp", "fdtd_kernels.hip", "fdtd_debye.hip", "fdtd_static.hip", "sur_host.cpp", "sur_kernels.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", os.path.join(PKG, "..", "include")]


def build(verbose: bool = False) -> str:
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    cmds = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        cmds.append([HIPCC] + FLAGS + ["-c", os.path.join(HERE, src), "-o", obj])
        objs.append(obj)
    procs = []
    for cmd in cmds:  # one compiler process per translation unit, in parallel
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
    bad = [cmd for cmd, p in zip(cmds, procs) if p.wait() != 0]
    if bad:
        raise subprocess.CalledProcessError(1, bad[0])
    tmp = OUT + ".tmp"
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
