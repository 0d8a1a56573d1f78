"""The oracle under AddressSanitizer, UndefinedBehaviorSanitizer and
LeakSanitizer, on the CPU: tests/sanitize_oracle.c calls every exported
oracle routine on small systems (a periodic crystal, a slab with a free axis
and a laser source, a chain for the two-temperature bar), with OpenMP on; an
invalid access, an undefined operation or a leak fails the run."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "sanitize_oracle.c")


def test_oracle_is_clean_under_the_sanitizers():
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "sanitize_oracle")
        build = subprocess.run(
            [gcc, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer", "-fopenmp", "-ffp-contract=off", SRC, "-lm", "-o", exe],
            capture_output=True, text=True, timeout=300)
        if build.returncode != 0 and "asan" in build.stderr.lower():
            pytest.skip("sanitizer runtime not available: " + build.stderr[-300:])
        assert build.returncode == 0, build.stderr[-3000:]
        env = dict(os.environ, OMP_NUM_THREADS="4", ASAN_OPTIONS="detect_leaks=1",
                   UBSAN_OPTIONS="print_stacktrace=1")
        run = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
        assert run.returncode == 0, (run.stdout + run.stderr)[-4000:]
        assert "sanitize_oracle: ok" in run.stdout
