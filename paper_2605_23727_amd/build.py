"""Build the gfx950 shared library ``libbs32.so`` in-tree with hipcc.

Usage: ``python -m paper_2605_23727_amd.build`` (or ``build()`` from Python).
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbs32.so")
SOURCES = ["bs32_mlp.hip", "bs32_lco.hip", "bs32_blas.cpp", "bs32_capi.cpp"]
# bs32_kernels.hip compiles as KERNEL_PARTS units, each instantiating its own kernel families
KERNEL_PARTS = 9
# hipBLASLt: the plain library product of 16-bit shared-coupling ensembles
LIBS = ["-L/opt/rocm/lib", "-lhipblaslt", "-Wl,--no-undefined"]

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=off",  # stage combinations evaluated exactly as written; FMAs only where spelled out
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def _compile(hipcc: str, unit: tuple, verbose: bool) -> str:
    src, part = unit
    stem = os.path.splitext(src)[0] + ("" if part is None else f"_p{part}")
    obj = os.path.join(CSRC, stem + ".o")
    defs = [] if part is None else [f"-DBS32_PART={part}"]
    cmd = [hipcc, *FLAGS, *defs, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{msg}")
    if msg.strip() and verbose:
        print(msg)
    return obj


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    # the translation units compile independently: one hipcc process each
    units = [("bs32_kernels.hip", p) for p in range(KERNEL_PARTS)] + [(src, None) for src in SOURCES]
    workers = max(1, min(len(units), os.cpu_count() or 1, 16))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(lambda u: _compile(hipcc, u, verbose), units))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, *LIBS, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
