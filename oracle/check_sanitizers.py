"""Run the oracle's CPU tests against the oracle built with AddressSanitizer
and UndefinedBehaviorSanitizer (host code only; the HIP library is not
involved).  Any invalid access, leak-free use-after-free, overflow or
undefined operation in ``lbfss_oracle.c`` aborts the run.

Usage: ``python oracle/check_sanitizers.py [pytest args]`` (default: every
``tests/test_oracle_*.py`` and ``tests/test_linear_theory.py``).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

from oracle import build  # noqa: E402


def runtime(name):
    return subprocess.run(["gcc", f"-print-file-name={name}"], check=True, capture_output=True,
                          text=True).stdout.strip()


def main(args):
    build.build(verbose=True, sanitize=True)
    env = dict(os.environ)
    env["LBFSS_ORACLE_SANITIZE"] = "1"
    # the interpreter is not instrumented: preload the runtimes, ignore its leaks
    env["LD_PRELOAD"] = ":".join([runtime("libasan.so"), runtime("libubsan.so")])
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    tests = args or sorted(os.path.join("tests", f) for f in os.listdir(os.path.join(ROOT, "tests"))
                           if f.startswith("test_oracle_") or f == "test_linear_theory.py")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider"] + tests
    print(" ".join(cmd), flush=True)
    return subprocess.run(cmd, cwd=ROOT, env=env).returncode


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
