"""Builds librtlbm.so (the HIP/C++ solver library) in-tree for gfx950.

    python paper_2609_23057_amd/build.py

Compiles the host setup and ABI layer as host C++ and the kernels as HIP for
gfx950, then links one shared library next to this file.  Packed-FP32
instructions are disabled for device code.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "librtlbm.so")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(ROOT, "include")]
# No automatic multiply-add contraction: the kernels write their fused
# multiply-adds explicitly, so every instantiation of a step rounds the same.
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-ffp-contract=off"]

SOURCES = [("rt_host.cpp", False), ("rt_abi.cpp", False), ("rt_kernels.hip", True), ("rt_sv.hip", True)]


def _compile(src, device):
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC] + COMMON
    if device:
        cmd += ["-x", "hip"] + DEVICE
    else:
        cmd += ["-D__HIP_PLATFORM_AMD__"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in (r.stderr or "").splitlines()
                    if "packed-fp32-ops" not in l)
    return obj, r.returncode, err, cmd


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        res = list(ex.map(lambda s: _compile(*s), SOURCES))
    for obj, rc, err, cmd in res:
        if rc != 0:
            raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), err))
        if verbose and err.strip():
            print(err, file=sys.stderr)
    link = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", OUT + ".tmp"] + \
        [r[0] for r in res]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(link), r.stderr))
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
