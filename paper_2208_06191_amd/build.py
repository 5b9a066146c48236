"""Builds the HIP library (libmbddc.so) in-tree for gfx950."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmbddc.so")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = True) -> str:
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    plan_o = os.path.join(bdir, "plan.o")
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-c", os.path.join(CSRC, "plan.cpp"), "-o", plan_o] + inc)
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    srv_o = os.path.join(bdir, "server.o")
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-pthread", "-D__HIP_PLATFORM_AMD__", "-I",
          os.path.join(rocm, "include"), "-c", os.path.join(CSRC, "server.cpp"), "-o", srv_o] + inc)
    dev_o = os.path.join(bdir, "mbddc.o")
    _run([hipcc] + HIP_FLAGS + inc + ["-c", os.path.join(CSRC, "mbddc.hip"), "-o", dev_o])
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", dev_o, plan_o, srv_o, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
