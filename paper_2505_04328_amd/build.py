"""Build libjd.so (the HIP kernels and the C ABI) in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libjd.so")
SOURCES = ["jd_kernels.hip", "fb_kernels.hip", "jd_api.cpp", "jd_feedback.cpp", "jd_server.cpp",
           "jd_noalloc.cpp", "jd_shapes.cpp"]
HEADERS = ["jd_device.hpp", "jd_launch.hpp", "jd_host.hpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("JD_OFFLOAD_ARCH", "gfx950")

# -ffp-contract=off: every FMA is written out, so the forward sweep and the
# recomputing adjoint evaluate bit-identical steps.  Packed FP32 instructions are
# disabled.
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas"]


def _obj(src: str) -> str:
    return os.path.join(CSRC, "_build", os.path.splitext(src)[0] + ".o")


def build(verbose: bool = False, jobs: int = 2) -> str:
    os.makedirs(os.path.join(CSRC, "_build"), exist_ok=True)
    procs = []
    t0 = time.time()
    for src in SOURCES:
        lang = ["-x", "hip"]
        cmd = [HIPCC, *lang, *FLAGS, "-c", os.path.join(CSRC, src), "-o", _obj(src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                            text=True)))
    for cmd, pr in procs:
        out, err = pr.communicate()
        if pr.returncode != 0:
            raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + err[-6000:])
        if verbose and err:
            sys.stderr.write(err[-3000:])
    link = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp",
            *[_obj(s) for s in SOURCES]]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + " ".join(link) + "\n" + r.stderr[-4000:])
    os.replace(LIB + ".tmp", LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s", flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
