"""Build libhdconv.so (gfx950) in-tree with hipcc.

Usage: ``python -m paper_2303_17510_amd.build`` or ``build()`` from Python.
Every source is compiled each call (the build is the "does it compile" check).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libhdconv.so")
BUILD_DIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("HDCONV_ARCH", "gfx950")

SOURCES = ["hd_k_fused.hip", "hd_k_lean.hip", "hd_k_batch.hip", "hd_k_multi.hip", "hd_k_outer.hip", "hd_mlp.hip", "hd_api.cpp", "hd_plan.cpp"]
# the two largest kernel files compile as two objects each (FP32 / FP64
# instances, selected by HD_PART), so the parallel build is not held up by them
SPLIT = {"hd_k_fused.hip", "hd_k_lean.hip", "hd_k_batch.hip", "hd_k_multi.hip"}
UNITS = [(s, part) for s in SOURCES for part in ((1, 2) if s in SPLIT else (0,))]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _flags():
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
            # packed FP32 instructions are kept out of generated code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I" + os.path.join(HERE, "..", "include")]


def _fresh(obj: str, src: str) -> bool:
    if not os.path.exists(obj):
        return False
    t = os.path.getmtime(obj)
    deps = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    deps += [os.path.join(CSRC, src), os.path.join(HERE, "..", "include", "hdconv.h")]
    return all(os.path.getmtime(d) < t for d in deps if os.path.exists(d))


def _compile(unit, verbose: bool, incremental: bool = False) -> str:
    src, part = unit
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ("_p%d" % part if part else "") + ".o")
    if incremental and _fresh(obj, src):
        return obj
    defs = ["-DHD_PART=%d" % part] if part else []
    cmd = [hipcc()] + _flags() + defs + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s%s" % (src, r.stdout, r.stderr))
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if err and verbose:
        print(err, file=sys.stderr)
    return obj


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (``incremental``: only those older than a header or source)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(UNITS), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda u: _compile(u, verbose, incremental), UNITS))
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed\n%s%s" % (r.stdout, r.stderr))
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv))
