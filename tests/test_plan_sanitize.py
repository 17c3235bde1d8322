"""The geometry plan builder (host C++) under AddressSanitizer and
UndefinedBehaviorSanitizer: every LED count of the workloads at 64, 128 and
256 px with and without darkfield, the 512 px plan with 16 + 32 LEDs, and a
geometry that must be rejected.  CPU only;
skipped when no host compiler is available."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.timeout(600)
def test_plan_builder_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = tmp_path / "plan_sanitize"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "native", "plan_sanitize.cpp"),
           os.path.join(ROOT, "paper_2407_20469_amd", "csrc", "plan.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=500)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "built" in r.stdout
