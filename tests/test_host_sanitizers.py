"""The library's host planning code (partition, setup plan, coarse space)
built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer and run
on seeded systems: no out-of-bounds access, use after free, leak or
undefined behaviour on the host side.  CPU only."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from workloads.mac_oseen import make_oseen_mac

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1104_3349_amd", "csrc")
SOURCES = [os.path.join(CSRC, f) for f in ("partition.cpp", "plan.cpp", "coarse.cpp")]
DRIVER = os.path.join(ROOT, "tests", "host", "sanitize_driver.cpp")

SYSTEMS = [dict(n=16, nu=0.1, m=4, sz=64, stretch=None), dict(n=48, nu=0.005, m=6, sz=40, stretch=1.05),
           dict(n=40, nu=0.01, m=9, sz=24, stretch=1.2), dict(n=64, nu=0.01, m=1, sz=100, stretch=None)]


def _write(path, rp, ci, v, m, sz):
    with open(path, "wb") as f:
        np.array([len(rp) - 1, len(ci), m, sz], dtype=np.int32).tofile(f)
        rp.astype(np.int32).tofile(f)
        ci.astype(np.int32).tofile(f)
        v.astype(np.float64).tofile(f)


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the ROCm headers")
def test_host_planning_under_sanitizers(tmp_path):
    exe = str(tmp_path / "drv")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, *SOURCES, DRIVER, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    files = []
    for q, c in enumerate(SYSTEMS):
        rp, ci, v, b, meta = make_oseen_mac(c["n"], c["nu"], stretch=c["stretch"], seed=q + 1)
        path = str(tmp_path / f"sys{q}.bin")
        _write(path, rp, ci, v, c["m"], c["sz"])
        files.append(path)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, *files], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    lines = [ln for ln in r.stdout.splitlines() if "plans" in ln]
    assert len(lines) == len(SYSTEMS)
    assert all(int(ln.split("plans ")[1].split()[0]) > 0 for ln in lines)
