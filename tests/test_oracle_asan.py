"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host C
code only): oracle/asan_driver.c runs every entry point on small hierarchies
of each kind (single level, harmonic rule, Galerkin, hybrid, truncated with
flexible CG, plain) and must finish clean."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_is_clean_under_asan_and_ubsan():
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_asan")
        cmd = [gcc, "-O1", "-g", "-std=c99", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-fno-omit-frame-pointer", "-fopenmp", os.path.join(ROOT, "oracle", "gmg_oracle.c"),
               os.path.join(ROOT, "oracle", "asan_driver.c"), "-lm", "-o", exe]
        b = subprocess.run(cmd, capture_output=True, text=True)
        if b.returncode != 0:
            pytest.skip(f"sanitizer build unavailable: {b.stderr[-300:]}")
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", OMP_NUM_THREADS="2")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
