"""The oracle's pin tests again, against a build instrumented with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc, host code only).

Any out-of-bounds access, use after free, signed overflow, misaligned access or other
undefined behaviour in the oracle's C code aborts the child process, so the pins pass
only if the oracle's arithmetic is also free of those faults.  The child runs with the
ASan runtime preloaded, since the interpreter itself is not instrumented; leak checking
is off (the interpreter keeps its own allocations until exit).
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_TESTS = ["test_oracle_prng_sprinkle.py", "test_oracle_matrix.py", "test_oracle_histogram.py",
             "test_oracle_action.py", "test_oracle_dalembertian.py", "test_oracle_chain.py",
             "test_oracle_ds2.py"]


def runtime(name: str) -> str:
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                          text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else ""


@pytest.mark.slow
def test_oracle_pins_under_asan_ubsan():
    asan = runtime("libasan.so")
    if not asan:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    env = dict(os.environ)
    env["ORACLE_SANITIZE"] = "1"
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = env.get("OMP_NUM_THREADS", "4")
    # build the instrumented library first, in this process's own environment
    build = subprocess.run([sys.executable, "-c", "import oracle; oracle.build(force=True)"],
                           cwd=ROOT, env={**env, "LD_PRELOAD": ""}, capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-3000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu and not slow", *[os.path.join("tests", t) for t in PIN_TESTS]],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout[-3000:] + r.stderr[-3000:])
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
