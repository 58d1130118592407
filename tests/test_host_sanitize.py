"""The planner and the host side of the C ABI under AddressSanitizer and
UndefinedBehaviorSanitizer.

hd_api.cpp and hd_plan.cpp are compiled again with the sanitizers on their
host code only (each -fsanitize= behind -Xarch_host; device code unchanged),
linked with the library's kernel objects and tests/sanitize/host_plan_check.cpp,
and run here without a GPU: thousands of host-only plans (1D/2D/3D, ordinary,
centered and Hermitian, forced inner form and whole rows, c64/c128, A = 2, 3),
the geometry entry points and invalid arguments.  Any sanitizer report fails
the run.
"""
import glob
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_2303_17510_amd")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
       "-fno-omit-frame-pointer"]


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.mark.timeout(600)
def test_host_paths_under_sanitizers(tmp_path):
    hipcc = _hipcc()
    objs = sorted(glob.glob(os.path.join(PKG, "_build", "hd_k_*.o")) + glob.glob(os.path.join(PKG, "_build", "hd_mlp.o")))
    if hipcc is None or not objs:
        pytest.skip("needs hipcc and the library's kernel objects (python -m paper_2303_17510_amd.build)")
    inc = ["-I" + os.path.join(ROOT, "include")]
    base = ["-O1", "-g", "-std=c++17", "-fPIC", "-Wno-unused-command-line-argument"]
    out = []
    for src in ("hd_api.cpp", "hd_plan.cpp"):
        o = str(tmp_path / (src + ".o"))
        cmd = [hipcc] + base + ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] \
            + inc + SAN + ["-x", "hip", "-c", os.path.join(PKG, "csrc", src), "-o", o]
        subprocess.run(cmd, check=True, capture_output=True)
        out.append(o)
    drv = str(tmp_path / "drv.o")
    subprocess.run([hipcc] + base + inc + SAN + ["-x", "c++", "-c", os.path.join(HERE, "sanitize", "host_plan_check.cpp"),
                    "-o", drv], check=True, capture_output=True)
    exe = str(tmp_path / "host_plan_check")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-fsanitize=address,undefined", "-fno-gpu-sanitize", drv] + out
                   + objs + ["-o", exe], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert r.stdout.strip().endswith("ok (0 failures)")
