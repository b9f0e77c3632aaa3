"""Both oracles built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only, no OpenMP) and run on tiny and degenerate lattices through
every entry point: no out-of-bounds access, no undefined behaviour, and the
Tau1 and LBGK forms still agree."""
import os
import shutil
import subprocess

import pytest

import oracle

HERE = os.path.dirname(oracle.__file__)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracles_under_sanitizers(tmp_path):
    exe = tmp_path / "sanitize_driver"
    build = subprocess.run(
        ["gcc", "-std=gnu99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         os.path.join(HERE, "sanitize_driver.c"), os.path.join(HERE, "tau1_oracle.c"),
         os.path.join(HERE, "tau1_oracle_2d.c"), "-o", str(exe), "-lm"],
        capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                         env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1"})
    assert run.returncode == 0, run.stdout + run.stderr
    assert run.stdout.strip() == "ok"
