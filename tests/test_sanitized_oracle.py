"""The oracle's CPU pins run once more against an AddressSanitizer +
UndefinedBehaviorSanitizer build of the oracle, in a child interpreter with the
sanitizer runtime preloaded: any out-of-bounds access, use after free or
undefined behaviour in the oracle aborts the child and fails this test."""

import os
import subprocess
import sys

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_asan_and_ubsan():
    lib = oracle.build(force=True, sanitize=True)
    asan = _runtime("libasan.so")
    assert asan, "gcc's AddressSanitizer runtime is missing"
    env = dict(os.environ, DBG_ORACLE_LIB=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    # the planted-mistake tests compile their own mutants and are left out
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
           "tests/test_oracle.py", "-k", "not planted_mistake"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr, tail
