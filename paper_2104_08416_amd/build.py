"""Build the gfx950 shared library ``libsem_hip.so`` in-tree with hipcc.

Usage: ``python -m paper_2104_08416_amd.build`` (or ``build()`` from Python). Always
recompiles. The host setup (``plan.cpp``) is compiled with ``-ffp-contract=off`` so the
centroid/cell arithmetic of the curve ordering is evaluated exactly as written.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsem_hip.so")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function"]
# Device code: no packed-FP32 VALU instructions (v_pk_*_f32), FP atomics in hardware.
DEVICE = [f"--offload-arch={ARCH}", "-mcode-object-version=5", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the HIP library)")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r.stdout


def build(verbose: bool = False) -> str:
    cc = hipcc()
    with tempfile.TemporaryDirectory(prefix="sem_build_") as tmp:
        objs = []
        jobs = [
            (os.path.join(CSRC, "plan.cpp"), COMMON + ["-ffp-contract=off"]),
            (os.path.join(CSRC, "tri.cpp"), COMMON + ["-ffp-contract=off"]),
            (os.path.join(CSRC, "kernels.hip"), COMMON + DEVICE + ["-x", "hip"]),
            (os.path.join(CSRC, "api.hip"), COMMON + DEVICE + ["-x", "hip"]),
        ]
        procs = []
        for src, flags in jobs:
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            cmd = [cc] + flags + ["-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd))
            procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                                text=True)))
            objs.append(obj)
        for cmd, pr in procs:
            out, _ = pr.communicate()
            if pr.returncode != 0:
                sys.stderr.write(out)
                raise RuntimeError("build step failed: " + " ".join(cmd))
            if verbose and out.strip():
                print(out)
        tmp_lib = LIB + ".tmp"
        _run([cc, f"--offload-arch={ARCH}", "-shared", "-o", tmp_lib] + objs)
        os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
