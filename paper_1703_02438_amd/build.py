"""Build libnumarck.so for gfx950 with hipcc (in-tree, next to this file).

Each HIP source is compiled to an object in parallel, then the objects are
linked into the shared library."""
from __future__ import annotations

import glob
import os
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnumarck.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=off: binary64 expressions are evaluated as written (no FMA),
# which the bit-exact results depend on.  Packed-FP32 instructions are
# disabled for all device code.
CFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fPIC", "-pthread",
]
LDFLAGS = ["--offload-arch=gfx950", "-fPIC", "-shared", "-pthread"]


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _run(cmd: list[str]) -> None:
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)


def build(verbose: bool = False) -> str:
    srcs = sources()
    with tempfile.TemporaryDirectory(prefix="nk_build_") as tmp:
        objs = [os.path.join(tmp, os.path.basename(s) + ".o") for s in srcs]
        cmds = [[HIPCC, *CFLAGS, "-c", s, "-o", o] for s, o in zip(srcs, objs)]
        jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            for f in [ex.submit(_run, c) for c in cmds]:
                f.result()
        tmp_lib = LIB + ".tmp"
        link = [HIPCC, *LDFLAGS, "-o", tmp_lib, *objs]
        _run(link)
        os.replace(tmp_lib, LIB)
        if verbose:
            for c in cmds + [link]:
                print(" ".join(c))
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
