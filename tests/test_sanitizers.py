"""The CPU test suite again with the oracle and the host code of librte built
under AddressSanitizer and UndefinedBehaviorSanitizer (`python -m
oracle.build --sanitize`, `python -m paper_1809_06417_amd.build --sanitize`;
`__graft_entry__.build()` makes both). The suite runs in a child process with
clang's shared sanitizer runtime preloaded; any report aborts it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_cpu_suite_is_clean_under_asan_and_ubsan():
    from oracle import build as ob
    from paper_1809_06417_amd import build as hb
    if not (os.path.exists(ob.SAN_LIB) and os.path.exists(hb.SAN_LIB)):
        pytest.skip("sanitizer builds absent (run __graft_entry__.build())")
    env = dict(os.environ, RTE_SANITIZE="1", LD_PRELOAD=ob.asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-m", "not gpu", "-q", "-x",
           "-p", "no:cacheprovider", "-k", "not test_cpu_suite_is_clean_under_asan_and_ubsan"]
    r = subprocess.run(cmd, env=env, cwd=ROOT, capture_output=True, text=True, timeout=1500)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
    assert " passed" in r.stdout, tail
