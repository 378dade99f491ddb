"""Build the FP64 CPU oracle (test infrastructure) into ``oracle/liboracle.so``.

Plain C11 compiled by gcc with ``-O2 -ffp-contract=off`` (no fast-math, no FMA
contraction) and OpenMP over chunks of paths.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "jd_oracle.c"), os.path.join(HERE, "fb_oracle.c")]
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-fopenmp", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(src=SRC, out: str = LIB, extra: list | None = None, quiet: bool = True) -> str:
    """Compile `src` (one path or a list of C files) into the shared library `out`."""
    srcs = [src] if isinstance(src, str) else list(src)
    # a private temporary name: concurrent builds (parallel test workers) each
    # rename a complete library into place
    tmp = f"{out}.{os.getpid()}.tmp"
    cmd = ["gcc", *CFLAGS, *(extra or []), "-o", tmp, *srcs, "-lm"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("oracle build failed:\n" + " ".join(cmd) + "\n" + res.stderr)
    if res.stderr and not quiet:
        sys.stderr.write(res.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(quiet=False))
