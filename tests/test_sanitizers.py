"""Address and undefined-behaviour sanitizer runs of the host code that checks the GPU path: the
oracle (oracle/oracle.cpp) and the input generator's native helpers (synth/_synth.cpp), built
with g++ -fsanitize=address,undefined and driven through every exported function on small
inputs, edge cases and error paths (tests/sanitize/driver.cpp, which also checks a hand-computed
factor). CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_and_generator_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "driver")
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
             "-ffp-contract=off", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    srcs = [os.path.join(ROOT, "tests", "sanitize", "driver.cpp"),
            os.path.join(ROOT, "oracle", "oracle.cpp"), os.path.join(ROOT, "synth", "_synth.cpp")]
    r = subprocess.run(["g++"] + flags + ["-o", exe] + srcs, capture_output=True, text=True)
    if r.returncode != 0 and ("asan" in r.stderr.lower() or "ubsan" in r.stderr.lower()):
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(run.stdout)
    assert run.returncode == 0, run.stderr[-4000:]
    assert "runtime error" not in run.stderr and "ERROR: AddressSanitizer" not in run.stderr
    assert "sanitized run ok" in run.stdout
