"""Host code and oracle under the compiler's sanitizers (CPU only).

The library's host source (argument checks, tuning table, packer, plans, the
allocation-free call, the host copy pool) is built with g++ against a
host-only stand-in for the HIP runtime (tests/native/fake_hip) whose kernel
launch checkers touch everything a launch may touch; the FP64 oracle is
built with gcc.  Each runs once with AddressSanitizer + UndefinedBehavior-
Sanitizer and once with ThreadSanitizer; any report fails the test."""
from __future__ import annotations

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
ASAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
TSAN = ["-fsanitize=thread"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1", TSAN_OPTIONS="halt_on_error=1")


def _build_and_run(tmp_path, name, cmd_tail, flags, args):
    exe = str(tmp_path / name)
    r = subprocess.run(cmd_tail[:1] + flags + cmd_tail[1:] + ["-o", exe], capture_output=True,
                       text=True)
    if r.returncode != 0 and "sanitize" in r.stderr and "unrecognized" in r.stderr:
        pytest.skip("compiler without this sanitizer")
    assert r.returncode == 0, r.stderr[-3000:]
    run = subprocess.run([exe] + args, capture_output=True, text=True, env=ENV, timeout=600)
    out = run.stdout + run.stderr
    assert run.returncode == 0 and "ERROR: " not in out and "WARNING: ThreadSanitizer" not in out \
        and "runtime error" not in out, out[-4000:]
    return out


def _host_cmd():
    return ["g++", "-std=c++17", "-O1", "-g", "-Wno-subobject-linkage",
            "-I", os.path.join(NATIVE, "fake_hip"), "-I", os.path.join(ROOT, "include"),
            "-I", os.path.join(ROOT, "paper_2604_06602_amd", "csrc"),
            os.path.join(NATIVE, "host_checks.cpp"), "-lpthread"]


def _oracle_cmd():
    return ["gcc", "-std=gnu99", "-O1", "-g", os.path.join(NATIVE, "oracle_checks.c"),
            os.path.join(ROOT, "oracle", "umi_oracle.c"), "-lm", "-lpthread"]


@pytest.mark.parametrize("flags,rounds", [(ASAN, "300"), (TSAN, "20")], ids=["asan_ubsan", "tsan"])
def test_host_code_under_sanitizers(tmp_path, flags, rounds):
    out = _build_and_run(tmp_path, "host_checks", _host_cmd(), flags, [rounds])
    assert "host checks ok" in out


@pytest.mark.parametrize("flags,rounds", [(ASAN, "15"), (TSAN, "4")], ids=["asan_ubsan", "tsan"])
def test_oracle_under_sanitizers(tmp_path, flags, rounds):
    out = _build_and_run(tmp_path, "oracle_checks", _oracle_cmd(), flags, [rounds])
    assert "oracle checks ok" in out
