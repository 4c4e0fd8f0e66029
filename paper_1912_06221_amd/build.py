"""Build the HIP/C++ library libardg.so in-tree for gfx950.

Host setup code (refops.cpp, meshsetup.cpp) and the C ABI (api.cpp) are plain
C++ compiled with g++; the kernels (kernels*.hip) are compiled by hipcc for
gfx950 with packed FP32 instructions disabled.  Everything is linked by hipcc
into one shared library next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libardg.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = os.environ.get("ARDG_OFFLOAD_ARCH", "gfx950")

HIP_DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmds):
    procs = [(c, subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)) for c in cmds]
    failed = []
    for c, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append((c, out.decode(errors="replace")))
    if failed:
        msg = "\n\n".join(" ".join(c) + "\n" + o for c, o in failed)
        raise RuntimeError("build failed:\n" + msg)


def build(verbose: bool = False) -> str:
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    os.makedirs(BUILD, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", f"-I{INCLUDE}", f"-I{CSRC}"]
    host = ["g++"] + common + ["-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include"]
    objs = []
    cmds = []
    for src in ("refops.cpp", "meshsetup.cpp", "api.cpp"):
        obj = os.path.join(BUILD, src.replace(".cpp", ".o"))
        cmds.append(host + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in ("kernels.hip", "kernels_mfma.hip", "kernels_edge_mfma.hip", "kernels_tensor.hip", "kernels_ns.hip", "noalloc.hip"):
        kobj = os.path.join(BUILD, src.replace(".hip", ".o"))
        cmds.append([hipcc, f"--offload-arch={ARCH}"] + common + HIP_DEVICE_FLAGS +
                    ["-c", os.path.join(CSRC, src), "-o", kobj])
        objs.append(kobj)
    _run(cmds)
    tmp = LIB + ".tmp"
    _run([[hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs +
          [f"-L{ROCM}/lib", "-lamdhip64"]])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
