"""Sanitizer runs of the host code on the CPU (no GPU needed):

* the oracle's C core under AddressSanitizer + UndefinedBehaviorSanitizer;
* the library's host-side schedule builders (threaded) under ASan + UBSan, built
  host-only from the library's own sources;
* the task-graph executor under ThreadSanitizer and under ASan + UBSan, built
  against a stand-in HIP header (streams, copies and pinned memory on the host),
  with CPU and GPU-domain workers and the inference pipeline.

Every driver checks its own results and prints "all ok"; a sanitizer report
makes it exit nonzero (recovery is off)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2004_10908_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           TSAN_OPTIONS="halt_on_error=1")


def run(exe, timeout=300):
    p = subprocess.run([exe], capture_output=True, text=True, timeout=timeout, env=ENV)
    out = p.stdout + p.stderr
    assert p.returncode == 0, out[-4000:]
    assert "all ok" in p.stdout, out[-4000:]
    assert "runtime error" not in out and "Sanitizer" not in out, out[-4000:]
    return out


def compile_(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert p.returncode == 0, p.stderr[-4000:]


def test_oracle_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    compile_(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "sdnn_oracle.c"),
              os.path.join(HERE, "oracle_driver.c"), "-o", exe, "-lm"])
    run(exe)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc is not installed")
def test_schedule_builders_asan_ubsan(tmp_path):
    exe = str(tmp_path / "sched_asan")
    compile_([HIPCC, "-x", "hip", "--offload-host-only", "-std=c++17", "-O1", "-g",
              "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-sanitize-recover=all", "-I", INCLUDE, "-I", CSRC,
              os.path.join(CSRC, "sdnn_rowsched.hip"), os.path.join(CSRC, "sdnn_sched.hip"),
              "-x", "c++", os.path.join(HERE, "sched_driver.cc"), "-o", exe])
    run(exe)


@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_taskgraph_sanitized(tmp_path, san):
    exe = str(tmp_path / ("tg_" + san.replace(",", "_")))
    # a host-only C++ copy of the executor's source, built by the host compiler
    src = str(tmp_path / "sdnn_taskgraph_host.cc")
    shutil.copyfile(os.path.join(CSRC, "sdnn_taskgraph.hip"), src)
    compile_(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=" + san,
              "-fno-sanitize-recover=all", "-DSDNN_TG_STANDIN_HIP", "-I", os.path.join(HERE, "standin"),
              "-I", INCLUDE, src, os.path.join(HERE, "taskgraph_driver.cc"), "-o", exe, "-lpthread"])
    out = run(exe)
    assert "rep 5:" in out
