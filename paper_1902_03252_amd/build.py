"""Build the gfx950 HIP library liblens.so in-tree with hipcc.

    python -m paper_1902_03252_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "liblens.so")
SOURCES = ["lens_kernels.hip", "lens_batched.hip", "lens_backward.hip", "lens_api.hip", "lens_tune.hip", "lens_mixed.hip", "lens_sampler.hip", "lens_nfw.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def flags() -> list[str]:
    return [
        "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
        # keep packed FP32 (v_pk_*_f32) out of the generated code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", INCLUDE, "-I", CSRC,
        "-Wall", "-Wno-unused-function",
    ]


# The packed-FP32 feature flag reaches hipcc's host pass too, which does not
# know it and says so once per source file; the device pass honours it.  Those
# lines are dropped from the log, everything else is shown.
_NOISE = "'-packed-fp32-ops' is not a recognized feature for this target (ignoring feature)"


def _run(cmd: list[str], verbose: bool) -> None:
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    rest = [ln for ln in (res.stdout + res.stderr).splitlines() if ln.strip() and ln.strip() != _NOISE]
    if res.returncode != 0:
        sys.stderr.write("\n".join(rest) + "\n")
        raise RuntimeError("hipcc failed: " + " ".join(cmd[-3:]))
    if verbose and rest:
        sys.stderr.write("\n".join(rest) + "\n")


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), then link liblens.so."""
    from concurrent.futures import ThreadPoolExecutor
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    cmds = [[hipcc()] + flags() + ["-c", "-o", o, os.path.join(CSRC, s)] for s, o in zip(SOURCES, objs)]
    jobs = max(1, min(len(cmds), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = LIB + ".tmp"
    _run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs, verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
