"""The oracle and the input generator under AddressSanitizer and UndefinedBehaviorSanitizer.

Both C libraries are built a second time with -fsanitize=address,undefined (host code,
gcc, errors fatal) and the oracle's pin tests run in a child Python process that loads
those builds (MAPCORE_ORACLE_LIB, MAPCORE_SYNTH_LIB) with the ASan runtime preloaded.  An
out-of-bounds access, use after free, signed overflow, misaligned access or other
undefined behaviour in either library aborts the child and fails this test.
"""
import glob
import os
import subprocess
import sys

import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    try:
        p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True, check=True)
    except (OSError, subprocess.CalledProcessError):
        return None
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.skipif(_asan_runtime() is None, reason="gcc has no AddressSanitizer runtime")
def test_oracle_pins_under_sanitizers():
    olib = oracle.build(variant="san")
    slib = synth.build_lib(sanitize=True)
    files = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    assert files
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": _asan_runtime(),
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "MAPCORE_ORACLE_LIB": olib,
        "MAPCORE_SYNTH_LIB": slib,
    })
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        *files, os.path.join(ROOT, "tests", "test_abi.py") + "::test_generated_mc_table_matches_oracle_rule"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "failed" not in r.stdout, tail
