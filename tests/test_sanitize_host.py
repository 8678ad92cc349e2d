"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU, no GPU call).

hinv_host.hip (every host-side entry point, plan builder and table check) is compiled with both
sanitizers on its host pass; the kernels' objects are the regular build.  tests/sanitize_driver.cpp,
linked with the sanitizer runtime, drives the host-only entry points (network assembly, workspace
sizing of every engine and precision, which builds and bounds-checks every engine plan, three-phase
assembly, and the argument-validation paths) over networks written here.  Any memory error, leak of
the library's own allocations or undefined behaviour aborts the driver with a report.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2105_10661_amd import build as hbuild
from paper_2105_10661_amd import cases

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
       "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _write(net, path):
    with open(path, "wb") as f:
        np.array([net.n_bus, net.n_branch, len(net.src_bus), len(net.parent)], np.int32).tofile(f)
        np.array([net.dt, net.freq], np.float64).tofile(f)
        for a, t in ((net.frm, np.int32), (net.to, np.int32), (net.R, np.float64), (net.L, np.float64),
                     (net.C, np.float64), (net.src_bus, np.int32), (net.src_amp, np.float64),
                     (net.src_phase, np.float64), (net.parent, np.int32), (net.bus_leaf, np.int32)):
            np.ascontiguousarray(a, t).tofile(f)


@pytest.mark.timeout(600)
def test_host_code_under_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("hipcc / clang++ not installed")
    if not os.path.exists(os.path.join(hbuild.OBJ, "k_panel.o")):
        hbuild.build()
    obj = str(tmp_path / "hinv_host_san.o")
    subprocess.check_call([HIPCC, *hbuild.FLAGS[:1], "-O1", "-g", "-std=c++17", "-fPIC", *hbuild.FLAGS[4:], *SAN,
                           "-c", os.path.join(hbuild.CSRC, "hinv_host.hip"), "-o", obj])
    drv = str(tmp_path / "driver.o")
    subprocess.check_call([CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "include"), "-c", os.path.join(ROOT, "tests", "sanitize_driver.cpp"),
                           "-o", drv])
    kernels = [os.path.join(hbuild.OBJ, s.replace(".hip", ".o")) for s in hbuild.SOURCES if s != "hinv_host.hip"]
    exe = str(tmp_path / "driver")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                           "-fsanitize=undefined", drv, obj, *kernels, "-o", exe])
    nets = {"net179": cases.net_179(), "ring716": cases.net_ring(4, 7), "ring1432": cases.net_ring(8, 4),
            "fine358": cases.net_ring_fine(2, 6)}
    files = []
    for name, net in nets.items():
        files.append(str(tmp_path / f"{name}.bin"))
        _write(net, files[-1])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, *files], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "checks passed" in r.stdout
    shutil.rmtree(tmp_path, ignore_errors=True)
