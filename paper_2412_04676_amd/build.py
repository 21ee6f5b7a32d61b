"""Build libbsdmrg.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libbsdmrg.so")
SOURCES = ["algebra.cpp", "blocks.cpp", "hpsi.cpp", "capi.cpp", "gemm.hip", "planes.hip", "serializer.hip", "davidson.hip", "truncate.hip", "stvec.cpp"]
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-mllvm", "-amdgpu-mfma-vgpr-form",
         "-Wno-unused-result", "-I" + os.path.join(os.path.dirname(HERE), "include")]


JOBS = min(8, os.cpu_count() or 1)


def _wait(job):
    cmd, proc = job
    if proc.wait() != 0:
        raise subprocess.CalledProcessError(proc.returncode, cmd)


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(objdir, src + ".o")
        cmd = [hipcc, "-x", "hip", "-c", path, "-o", obj] + [f for f in FLAGS if f != "-shared"]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
        if len(procs) >= JOBS:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    tmp = OUT + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
