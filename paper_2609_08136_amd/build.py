"""Builds libnys.so (the HIP library behind the C ABI in include/nys.h) for gfx950.

The tile instantiations and their dispatch are generated first (csrc/gen_dispatch.py,
into the build directory); they and every HIP source under csrc/ are compiled by hipcc
in parallel and linked into paper_2609_08136_amd/libnys.so, next to this file.  Run as a
module (`python -m paper_2609_08136_amd.build`) or call build().
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
GEN = os.path.join(OBJ, "gen")
LIB = os.path.join(HERE, "libnys.so")

sys.path.insert(0, CSRC)
import gen_dispatch  # noqa: E402

# every HIP source of csrc/ is one translation unit of the library, and so is every
# generated dispatch source (written into GEN by build())
SOURCES = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                 if f.endswith(".hip") and f not in gen_dispatch.GENERATED)

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
# Packed FP32 VALU instructions are disabled for every device compile.
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
]


def _compile(src: str) -> str:
    out = os.path.join(OBJ, os.path.splitext(os.path.basename(src))[0] + ".o")
    cmd = [HIPCC, *CFLAGS, "-I", CSRC, "-c", src, "-o", out]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stderr[-6000:]}")
    return out


def build(jobs: int | None = None, verbose: bool = True) -> str:
    """Generate the dispatch sources, compile everything and link libnys.so; returns the
    library path."""
    os.makedirs(OBJ, exist_ok=True)
    sources = SOURCES + gen_dispatch.write_all(GEN)
    jobs = jobs or min(len(sources), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    # largest translation units first
    order = sorted(sources, key=lambda s: -os.path.getsize(s))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, order))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lrocblas"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr[-4000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
