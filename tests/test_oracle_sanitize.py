"""The oracle built under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only; gcc), driven through every entry point on small inputs by
oracle/sanitize_driver.c: whole steps on a ragged grid, an empty particle set,
a one-cell grid, reseeding, the surface field and marching cubes. Any
out-of-bounds access, leak or undefined behaviour aborts the driver."""
import os
import shutil
import subprocess

import pytest

ORACLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "orc_sanitize")
    cmd = ["gcc", "-std=c99", "-g", "-O1", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-o", exe, os.path.join(ORACLE, "sanitize_driver.c"), os.path.join(ORACLE, "flip_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    # verify_asan_link_order=0: a library preloaded by the environment may come first
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
