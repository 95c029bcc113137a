"""The oracle's C code under AddressSanitizer (with its leak checker) and
UndefinedBehaviorSanitizer, host only: `oracle_sanitize_driver.c` calls
every entry point on small 1D/2D/3D grids with every boundary kind,
splitting, switch mode and weighting, and the refusals of invalid
arguments; any out-of-bounds access, use after free, leak or undefined
operation ends the run with an error.  (Built without OpenMP: the loops
then run on one thread, the same arithmetic.)"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")
SOURCES = ["weno_scalar.c", "charsys.c", "face.c", "solver.c"]


def test_oracle_clean_under_address_and_undefined_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_sanitize")
    cmd = [gcc, "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", ORACLE, "-o", exe]
    cmd += [os.path.join(ORACLE, s) for s in SOURCES]
    cmd += [os.path.join(HERE, "oracle_sanitize_driver.c"), "-lm"]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    if b.returncode != 0 and "asan" in (b.stderr or "").lower() and "cannot find" in b.stderr:
        pytest.skip("the sanitizer runtimes are not installed")
    assert b.returncode == 0, b.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout[-1000:], r.stderr[-3000:])
    assert "oracle under sanitizers: ok" in r.stdout
