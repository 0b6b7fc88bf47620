"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only): oracle.c and a
small C driver (tests/sanitize_oracle_main.c) are built with -fsanitize=address,undefined and
every routine runs on ragged tiny grids; any memory error, leak or undefined operation fails
the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    subprocess.check_call(["gcc", "-O1", "-g", "-ffp-contract=off", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-Wall", "-o", exe,
                           os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "tests", "sanitize_oracle_main.c"),
                           "-lm"])
    # verify_asan_link_order=0: the runtime need not come first when the environment preloads
    # other libraries
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ERROR" not in r.stderr and "runtime error" not in r.stderr, r.stderr
