"""Build libhgks.so (HIP kernels for gfx950 + host C ABI) in-tree.

    python -m paper_2304_09485_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libhgks.so")
ARCH = os.environ.get("HGKS_OFFLOAD_ARCH", "gfx950")

# packed FP32 VALU instructions are disabled for all device code
HIPFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src, kind in (("hgks_kernels.hip", "hip"), ("hgks_api.cpp", "hip"), ("hgks_server.cpp", "hip"),
                      ("mesh_prep.cpp", "cxx")):
        obj = os.path.join(BUILD, src + ".o")
        path = os.path.join(CSRC, src)
        if kind == "hip":
            _run(["hipcc", *HIPFLAGS, "-c", path, "-o", obj])
        else:
            _run(["g++", "-O2", "-std=c++17", "-fPIC", "-fopenmp", "-I", CSRC, "-c", path, "-o", obj])
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lgomp"])
    os.replace(tmp, LIB)
    # operation count of the flux per Gauss point (host instantiation of the
    # same template with a counting scalar), used by the roofline report
    exe = os.path.join(BUILD, "flopcount")
    _run(["hipcc", "-O1", "-std=c++17", "-I", CSRC, os.path.join(CSRC, "flopcount.cpp"), "-o", exe])
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    with open(os.path.join(HERE, "flux_flops.json"), "w") as f:
        f.write(out)
    # host instantiation of the flux for the CPU tests (not part of libhgks)
    _run(["hipcc", "-O2", "-std=c++17", "-fPIC", "-shared", "-I", CSRC, os.path.join(CSRC, "host_check.cpp"),
          "-o", HOSTCHECK])
    return LIB


HOSTCHECK = os.path.join(BUILD, "libhgks_hostcheck.so")


if __name__ == "__main__":
    build()
    sys.exit(0)
