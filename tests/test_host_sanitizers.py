"""The host code of every library source under AddressSanitizer and
UndefinedBehaviorSanitizer (host side only; the device code is compiled as
usual and never runs): tests/native/host_checks.cpp drives the C ABI's host
paths -- tables, workspace sizing, validation of seeded random arguments,
plan and batch creation and destruction over a placeholder address -- with
leak detection on.  No GPU is touched."""

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1401_7824_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_SOURCES = ["runtime.hip", "batch.hip", "mg_kernels.hip", "mg_tiles.hip", "sdc_kernels.hip", "compact.hip",
               "mlsdc.hip"]
# sanitizers on the host code only: each one directly after -Xarch_host
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


def _run(cmd):
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert res.returncode == 0, " ".join(cmd) + "\n" + res.stdout[-4000:]


@pytest.mark.slow
@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    out = str(tmp_path)
    common = ["-O1", "-g", "-fPIC", "-std=c++17", "-I", INCLUDE, "-fno-omit-frame-pointer"]
    jobs = []
    objs = []
    for src in HIP_SOURCES:
        o = os.path.join(out, src + ".o")
        jobs.append([HIPCC, "--offload-arch=gfx950"] + common + HOST_SAN +
                    ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
                     "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    o = os.path.join(out, "tables.o")
    jobs.append(["g++"] + common + ["-fsanitize=address,undefined", "-c", os.path.join(CSRC, "tables.cpp"), "-o", o])
    objs.append(o)
    o = os.path.join(out, "host_checks.o")
    jobs.append([HIPCC] + common + HOST_SAN +
                ["-c", "-x", "c++", os.path.join(ROOT, "tests", "native", "host_checks.cpp"), "-o", o])
    objs.append(o)
    with ThreadPoolExecutor(min(8, len(jobs))) as ex:
        list(ex.map(_run, jobs))
    exe = os.path.join(out, "host_checks")
    _run([HIPCC, "-fsanitize=address,undefined", "-o", exe] + objs)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout[-6000:]
    assert "host checks passed" in res.stdout
