"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only): oracle/sanitize_driver.c calls every oracle entry
point on small seeded matrices (mixed and empty block rows, rectangular
shapes, filters on both sides of zero, every sign order, the purifications,
the square-root iteration, the non-orthogonal density) and frees every
result; any out-of-bounds access, use after free, leak or undefined
behaviour ends the run with a sanitizer report and a non-zero status."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = tmp_path / "orc_san"
    src = os.path.join(ROOT, "oracle", "sanitize_driver.c")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fopenmp", "-ffp-contract=off",
           "-I", os.path.join(ROOT, "oracle"), "-o", str(exe), src, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr + r.stdout).lower():
        pytest.skip("gcc has no sanitizer runtime here")
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0")
    env.pop("LD_PRELOAD", None)
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "every call returned its expected status" in run.stdout
