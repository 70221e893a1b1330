"""The oracle's pins under AddressSanitizer and UndefinedBehaviorSanitizer:
oracle.c is built with both (host code only, gcc), and the oracle pin tests
run in a child process that loads that build (ORACLE_LIB) with the ASan
runtime preloaded.  Any out-of-bounds access, use after free, signed
overflow, misaligned or null access in the oracle aborts the child.  A copy
with a planted overflow (Algorithm 1 clearing one value past y) must be
caught, so the harness is known to watch the oracle's code."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")
PINS = ["tests/test_oracle.py", "tests/test_oracle_sell.py", "tests/test_oracle_mg.py"]


def _build(src, out):
    subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                    "-shared", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-o", out, src, "-lm"], check=True)


def _env(lib, asan):
    return dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=asan,
                ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
                UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.mark.slow
def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's ASan runtime is not installed")
    lib = str(tmp_path / "liboracle_san.so")
    _build(SRC, lib)
    # the harness catches a planted overflow (one value past y in Algorithm 1)
    bad_src = tmp_path / "oracle_bad.c"
    text = open(SRC).read()
    planted = text.replace("    for (int64_t i = 0; i < nrows; ++i)\n        y[i] = 0.0;\n",
                           "    for (int64_t i = 0; i <= nrows; ++i)\n        y[i] = 0.0;\n", 1)
    assert planted != text
    bad_src.write_text(planted)
    bad = str(tmp_path / "liboracle_bad.so")
    _build(str(bad_src), bad)
    probe = ("import numpy as np, oracle as o; "
             "o.coo_spmv(3, np.array([0, 2], np.int32), np.array([1, 2], np.int32), "
             "np.array([1.0, 2.0]), np.ones(3))")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=_env(bad, asan),
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "AddressSanitizer" in r.stderr, r.stderr[-2000:]
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=_env(lib, asan),
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    # the pins
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu and not slow",
                        "-p", "no:cacheprovider", *PINS], cwd=ROOT, env=_env(lib, asan),
                       capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
    assert " passed" in tail
