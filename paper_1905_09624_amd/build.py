"""Build the HIP library libcobs.so in-tree for gfx950 (hipcc, no JIT)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libcobs.so")
HIPCC = "/opt/rocm/bin/hipcc"
ARCH = os.environ.get("COBS_OFFLOAD_ARCH", "gfx950")

# packed-fp32 instructions are disabled for every HIP translation unit
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
          "-I", os.path.join(PKG, "..", "include")]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_SOURCES = ["lib.cpp", "query.cpp", "index_ops.cpp", "serve.cpp", "docset.cpp"]
DEVICE_SOURCES = ["kernels.hip", "gather.hip"]


def build(verbose: bool = False) -> str:
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    jobs = []
    for src in DEVICE_SOURCES:
        obj = os.path.join(objdir, src + ".o")
        jobs.append([HIPCC, *COMMON, *DEVICE, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in HOST_SOURCES:
        if not os.path.exists(os.path.join(CSRC, src)):
            continue
        obj = os.path.join(objdir, src + ".o")
        jobs.append([HIPCC, *COMMON, *DEVICE, "--cuda-host-only", "-c",
                     os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    procs = [subprocess.Popen(j, stdout=subprocess.PIPE, stderr=subprocess.STDOUT) for j in jobs]
    for j, p in zip(jobs, procs):
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(j)}\n{text}")
        if verbose and text.strip():
            print(text)
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, *DEVICE, "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
