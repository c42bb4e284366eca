"""AddressSanitizer + UndefinedBehaviorSanitizer run of the CPU oracle (test
infrastructure only, host code, gcc).

build() compiles oracle/rzo.c with -fsanitize=address,undefined into
oracle/librzo_san.so (any undefined behaviour aborts: no recovery).  run()
executes the oracle's CPU test files in a child interpreter that loads that
build (environment RZO_LIB) with the ASan runtime preloaded, and returns the
child's exit status and output.  `python oracle/sanitize.py` does both.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "librzo_san.so")


def build() -> str:
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off",
           "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fPIC", "-shared",
           os.path.join(HERE, "rzo.c"), "-o", LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def _runtime(name: str) -> str:
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True,
                         check=True).stdout.strip()
    return os.path.realpath(out)


def run(tests=None, timeout: float = 900.0):
    """Run the oracle test files (default: every tests/test_oracle_*.py) against
    the sanitized build.  Returns (returncode, combined output)."""
    if tests is None:
        tdir = os.path.join(ROOT, "tests")
        tests = sorted(os.path.join(tdir, f) for f in os.listdir(tdir)
                       if f.startswith("test_oracle_") and f.endswith(".py"))
    env = dict(os.environ)
    env["RZO_LIB"] = LIB
    env["LD_PRELOAD"] = _runtime("libasan.so")
    # the interpreter itself is not instrumented and keeps objects alive to
    # the end: leak reports would be about it, not the oracle
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    # --capture=sys leaves file descriptor 2 to the sanitizers' reports
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "--capture=sys",
           "-m", "not gpu", *tests]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=timeout)
    return r.returncode, r.stdout + r.stderr


if __name__ == "__main__":
    build()
    rc, out = run(sys.argv[1:] or None)
    sys.stdout.write(out)
    sys.exit(rc)
