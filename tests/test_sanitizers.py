"""The oracle's pins under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): the oracle is rebuilt with -fsanitize=address,undefined (every
finding fatal) and its two pin suites run in a child process with the ASan
runtime preloaded.  An out-of-bounds access, a use after free or undefined
arithmetic anywhere in the oracle's setup, cycle, solves, FCG and time step
fails this test."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.timeout(900)
def test_oracle_pins_under_asan_and_ubsan():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    oracle.build_sanitized()
    env = dict(os.environ)
    env.update(NN4MG_ORACLE_SANITIZED="1", LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_step_oracle.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=880)
    tail = (p.stdout[-3000:] + p.stderr[-3000:])
    assert p.returncode == 0, tail
    assert "passed" in p.stdout and "ERROR: AddressSanitizer" not in p.stderr and "runtime error" not in p.stderr, tail
