"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, any report is fatal) and driven through every entry point by
tests/oracle_sanitize_driver.c on small lattices: no out-of-bounds access,
leak, use after free, signed overflow or other undefined behaviour, and the
amounts conserved along the way (no GPU)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_sanitize_driver")
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fopenmp",
           "-ffp-contract=off", "-Wall", "-Wextra", "-Werror",
           os.path.join(HERE, "oracle_sanitize_driver.c"), os.path.join(ROOT, "oracle", "dsm_oracle.c"),
           "-lm", "-o", exe]
    subprocess.run(cmd, check=True, cwd=HERE)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "all checks passed" in r.stdout
