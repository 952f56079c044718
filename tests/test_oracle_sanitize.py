"""The CPU oracle (and the seeded input generator that feeds it) built with
AddressSanitizer and UndefinedBehaviorSanitizer and driven through every entry
point on small seeded inputs and on arbitrary codec records
(tests/sanitize_main.c).  Serial build (no OpenMP) so that the sanitizers see
one thread of each loop."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "sanitize_main"
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "tests", "sanitize_main.c"), os.path.join(ROOT, "oracle", "oracle.c"),
           os.path.join(ROOT, "volgen", "volgen.c"), "-o", str(exe), "-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert p.returncode == 0, p.stdout[-2000:] + p.stderr[-4000:]
    assert "sanitize ok" in p.stdout
