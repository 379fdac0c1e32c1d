"""Sanitizer runs on the CPU: the oracle and the library's host code under
the address and undefined-behaviour sanitizers, and the serving scheduler,
driven by several threads as the server drives it, under the thread
sanitizer.  Device code is never built with a sanitizer (the library's
checking build passes each flag to the host compilation only)."""
from __future__ import annotations

import os
import subprocess

import pytest

from paper_1701_05975_amd import build

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = os.path.join(HERE, "sanitize")


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(map(str, cmd))}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = tmp_path / "oracle_check"
    run(["gcc", "-std=c11", "-O1", "-g", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-pthread", os.path.join(ROOT, "oracle", "oracle.c"),
         os.path.join(SAN, "oracle_check.c"), "-o", str(exe), "-lm"])
    r = run([str(exe)], env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0"})
    assert "OK" in r.stdout


def test_host_library_under_address_and_undefined_sanitizers(tmp_path):
    lib = build.build(out=str(tmp_path / "libbcgpu_san.so"), objdir=str(tmp_path / "obj"),
                      sanitize=True)
    exe = tmp_path / "host_ingest_check"
    run([build.hipcc(), "-x", "c++", "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__",
         "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
         os.path.join(SAN, "host_ingest_check.cpp"), "-x", "none", lib, "-o", str(exe),
         f"-Wl,-rpath,{tmp_path}"])
    # leaks inside the HIP runtime are not this library's
    r = run([str(exe)], env={**os.environ, "ASAN_OPTIONS": "detect_leaks=0"})
    assert "OK" in r.stdout


def test_server_scheduling_under_thread_sanitizer(tmp_path):
    # ROCm's clang: its thread sanitizer sees the unlock inside a timed
    # condition-variable wait (pthread_cond_clockwait), which GCC 11's does not
    exe = tmp_path / "server_threads_check"
    clang = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(clang):
        pytest.skip("ROCm clang++ not found")
    run([clang, "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread",
         os.path.join(SAN, "server_threads_check.cpp"), "-o", str(exe)])
    r = run([str(exe)], env={**os.environ, "TSAN_OPTIONS": "halt_on_error=1"})
    assert "OK" in r.stdout
