"""AddressSanitizer + UndefinedBehaviorSanitizer build of the CPU oracle and
the seeded input generators (host code only; no GPU): tests/sanitize_driver.c
runs every generator and every oracle routine on small matrices of each kind,
and any out-of-bounds access, leak or undefined operation fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_and_generators_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "sanitize_driver")
    srcs = [os.path.join(ROOT, "tests", "sanitize_driver.c"), os.path.join(ROOT, "oracle", "spmv_oracle.c"),
            os.path.join(ROOT, "paper_1805_11938_amd", "synth", "synth.c")]
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wall", "-o", exe, *srcs, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, OMP_NUM_THREADS="3",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "all sanitizer cases passed" in r.stderr
