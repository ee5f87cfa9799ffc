"""Compiles libb2sr.so (all HIP sources under csrc/) for gfx950 with hipcc:
one object per source, compiled in parallel, then one link."""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libb2sr.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Wall", "-Wno-unused-function",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def build(verbose: bool = False, jobs: int | None = None, extra_flags: list[str] | None = None,
          out: str | None = None) -> str:
    """Builds the library (at `out`, default the package's libb2sr.so) with the
    standard flags plus `extra_flags`."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    lib = out or LIB
    flags = HIPCC_FLAGS + list(extra_flags or [])
    inc = ["-I", os.path.join(REPO, "include"), "-I", os.path.join(HERE, "csrc")]
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with tempfile.TemporaryDirectory(prefix="b2sr_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(src) + ".o") for src in srcs]

        def compile_one(pair):
            src, obj = pair
            cmd = [hipcc, *flags, *inc, "-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.run(cmd, check=True)

        with ThreadPoolExecutor(jobs) as pool:
            list(pool.map(compile_one, zip(srcs, objs)))
        tmp = lib + ".tmp"
        link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
