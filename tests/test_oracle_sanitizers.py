"""The oracle under the address and undefined-behaviour sanitizers (CPU).

A standalone driver (oracle/sanitize_main.c) includes the oracle source and
runs every step option, the outputs and the reference adjoint on small
lattices; built with gcc -fsanitize=address,undefined it must finish with
no sanitizer report and finite results."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    src = os.path.join(ROOT, "oracle", "sanitize_main.c")
    exe = os.path.join(tmp_path, "oracle_sanitized")
    build = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fno-fast-math",
             "-ffp-contract=off", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-I", os.path.join(ROOT, "oracle"), "-o", exe, src, "-lm"]
    subprocess.run(build, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in r.stderr
    assert "runtime error" not in r.stderr
    assert r.stdout.count(" ok") == 9, r.stdout
