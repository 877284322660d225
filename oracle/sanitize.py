"""AddressSanitizer + UndefinedBehaviorSanitizer run of the CPU oracle (test
infrastructure only, host code only).

    python -m oracle.sanitize            # build, then run the oracle's CPU tests

builds ``librbf_oracle_san.so`` from the same source with gcc
``-fsanitize=address,undefined`` (any UB report aborts the process) and runs
``pytest -m "not gpu" tests/test_oracle_*.py`` in a child process that
preloads the ASan runtime and loads the sanitized library in place of the
plain one (``RBF_ORACLE_LIB``).  Leak checking is off: the Python interpreter
itself keeps memory alive at exit.
"""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "rbf_oracle.c")
LIB = os.path.join(HERE, "librbf_oracle_san.so")


def build() -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-std=c11", "-Wall", "-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def run(pytest_args=()) -> int:
    lib = build()
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["RBF_ORACLE_LIB"] = lib
    tests = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu and not slow", "-p", "no:cacheprovider",
           *tests, *pytest_args]
    return subprocess.call(cmd, cwd=ROOT, env=env)


if __name__ == "__main__":
    sys.exit(run(sys.argv[1:]))
