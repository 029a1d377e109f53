"""The CPU oracle under sanitizers: every entry point on small seeded inputs and edge cases
(zero, saturating and huge LLRs, D = 1..256, L = 1..255, whole-code nodes) in a build with
AddressSanitizer and UndefinedBehaviorSanitizer, and concurrent batch calls on disjoint
frames (as the Python wrapper splits a batch) in a ThreadSanitizer build.  Host code only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "tests", "sanitize", "oracle_driver.cpp"),
       os.path.join(ROOT, "oracle", "polar_oracle.cpp")]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def _build_and_run(tmp_path, flags, args):
    exe = str(tmp_path / "driver")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer"] + flags +
                          ["-I" + os.path.join(ROOT, "oracle")] + SRC + ["-o", exe, "-lpthread"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe] + args, capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "oracle driver done" in r.stdout, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "WARNING" not in r.stderr, r.stderr[-4000:]


def test_oracle_address_and_undefined_behaviour_sanitizers(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"], [])


def test_oracle_thread_sanitizer_concurrent_batches(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=thread"], ["4"])
