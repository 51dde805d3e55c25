"""The request server's host logic under ThreadSanitizer (CPU only): six
threads submit, poll and wait concurrently on a fake-device server with a
small memory budget and injected failures; the binary must finish with every
request accounted for and no data race reported."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists("/opt/rocm/lib"),
                    reason="needs g++ and the ROCm host runtime")
def test_server_host_logic_is_race_free():
    tmp = tempfile.mkdtemp(prefix="mpdd_tsan_")
    try:
        exe = os.path.join(tmp, "server_tsan")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-D__HIP_PLATFORM_AMD__",
               "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
               os.path.join(ROOT, "tests", "tsan", "server_tsan_main.cpp"),
               os.path.join(ROOT, "paper_2109_13406_amd", "csrc", "server.cpp"),
               "-o", exe, "-L/opt/rocm/lib", "-lamdhip64", "-lpthread",
               "-Wl,-rpath,/opt/rocm/lib"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
        assert r.returncode == 0, (r.stdout, r.stderr[-2000:])
        assert "done=360 bad=0" in r.stdout
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
