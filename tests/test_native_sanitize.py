"""AddressSanitizer and UndefinedBehaviorSanitizer build of the library's host setup
(plan.cpp, tri.cpp) with g++, driven on quadrilateral and triangle meshes (jittered, graded,
every element order, both tilings). Host code only: no GPU code is built here."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2104_08416_amd", "csrc")


def _write(path, vxy, elems, c2, p):
    with open(path, "wb") as f:
        np.array([vxy.shape[0], elems.shape[0], elems.shape[1], p], np.int64).tofile(f)
        np.ascontiguousarray(vxy, np.float64).tofile(f)
        np.ascontiguousarray(elems, np.int32).tofile(f)
        np.ascontiguousarray(c2, np.float64).tofile(f)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not installed")
def test_plan_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "plan_sanitize")
    cmd = ["g++", "-std=gnu++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "tri.cpp"),
           os.path.join(ROOT, "tests", "native", "plan_sanitize.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    files = []
    for name, kw in (("layered1024", dict(n=9)), ("graded1414", dict(n=7, p=5)), ("tri2000", dict(n=8, p=5)),
                     ("tri2000", dict(n=6, p=1))):
        wl = workloads.workload(name, **kw)
        path = str(tmp_path / f"{name}_{wl.nx}_{wl.p}.bin")
        _write(path, wl.vxy, wl.quads, wl.c2, wl.p)
        files.append(path)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe] + files, capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.stdout.count("order") == 4 * 6 * 2
