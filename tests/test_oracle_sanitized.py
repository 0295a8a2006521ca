"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU).  A child interpreter loads the sanitizer build through MIBH_ORACLE_SO
with the ASan runtime preloaded and runs the oracle's own CPU tests (tree,
physics, refit, block steps); any out-of-bounds access, use after free or
undefined operation ends it with a report."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SUITES = ["tests/test_oracle_keys_tree.py", "tests/test_oracle_physics.py", "tests/test_oracle_refit.py",
          "tests/test_oracle_blockstep.py", "tests/test_oracle_leapfrog.py"]


def test_oracle_tests_pass_under_asan_and_ubsan():
    import oracle
    try:
        oracle.build_sanitized()
        env = oracle.sanitizer_env()
    except (subprocess.CalledProcessError, FileNotFoundError) as e:  # no sanitizer runtime in this toolchain
        pytest.skip(f"sanitizer build unavailable: {e}")
    env["OMP_NUM_THREADS"] = "4"
    # -s: a report has to reach stderr, not the capture file of the test that dies
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-s", "-p", "no:cacheprovider", "-m", "not gpu", *SUITES],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
