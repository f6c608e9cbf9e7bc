"""Memory and undefined-behaviour checks on the CPU: the oracle's test suite
run against an AddressSanitizer + UndefinedBehaviorSanitizer build of the
oracle, and libsrt's host-side tests against a sanitized build of its host
code (no device code: validation, workspace arithmetic, memory limit)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(env, args, timeout):
    # -s: a sanitizer report goes to the process's stderr, which pytest would
    # otherwise capture and lose when the sanitizer ends the process
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-s", "-p", "no:cacheprovider",
                        *args], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=timeout)
    assert r.returncode == 0, (r.stdout[-4000:] + "\n" + r.stderr[-4000:])
    return r.stdout


def test_oracle_suite_under_asan_and_ubsan(tmp_path):
    import oracle
    lib = oracle.build_sanitized(str(tmp_path / "liboracle_asan.so"))
    libasan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    env = dict(os.environ, SRT_ORACLE_LIB=lib, LD_PRELOAD=libasan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", SRT_ORACLE_THREADS="4")
    out = _run(env, ["-m", "not gpu", "tests/test_oracle.py"], 900)
    assert "passed" in out


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    from paper_2504_06598_amd import build
    lib = build.build_host_sanitized(str(tmp_path))
    env = dict(os.environ, SRT_LIB_PATH=lib, LD_PRELOAD=build.asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    out = _run(env, ["-m", "not gpu", "tests/test_library.py"], 600)
    assert "passed" in out
