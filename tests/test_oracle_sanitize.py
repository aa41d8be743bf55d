"""The oracle's pins again, on a build of oracle.c with AddressSanitizer and
UndefinedBehaviorSanitizer (any out-of-bounds access, use after free or
undefined arithmetic in the C oracle aborts the run).  CPU only."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle.py", "tests/test_oracle_lb.py", "tests/test_oracle_knn.py",
        "tests/test_oracle_wdtw.py", "tests/test_oracle_dba.py"]


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if p.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = tmp_path / "liboracle_san.so"
    subprocess.check_call(
        ["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-pthread",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
         "-o", str(lib), os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    env = dict(os.environ)
    env.update({"ORACLE_LIB": str(lib), "LD_PRELOAD": asan,
                # the interpreter itself keeps memory to the end: report
                # errors in the oracle, not the interpreter's leaks
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    p = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider", *PINS], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=900)
    tail = (p.stdout + p.stderr)[-4000:]
    assert p.returncode == 0, tail
    assert "passed" in p.stdout, tail
    assert "ERROR: AddressSanitizer" not in p.stderr and "runtime error" not in p.stderr, tail
