"""The request server's host logic (paper_2103_08932_amd/csrc/serve.hip) on the CPU: the real
source is compiled with g++ against a mock HIP runtime and mocked body / launch functions
(tests/server_mock/), with AddressSanitizer and UndefinedBehaviorSanitizer.  Random streams of 2D and
3D requests, some of which fail setup or hit their step limit, are served under tight and loose
memory budgets; every batched launch checks that each row it is given is the current table row of
a live, set-up body of the launch's dimension (a stale or permuted table would hand one body's
arrays to another body's kernels), and the server must complete every request."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MOCK = os.path.join(ROOT, "tests", "server_mock")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_server_host_logic_under_sanitizers(tmp_path):
    exe = str(tmp_path / "server_mock")
    cmd = ["g++", "-std=c++17", "-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           f"-I{MOCK}", f"-I{os.path.join(ROOT, 'paper_2103_08932_amd', 'csrc')}",
           "-x", "c++", os.path.join(ROOT, "paper_2103_08932_amd", "csrc", "serve.hip"),
           "-x", "c++", os.path.join(MOCK, "server_mock.cpp"), "-o", exe, "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", TLSPH_SERVE_GROUPS="4")
    r = subprocess.run([exe, "12"], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "mock server ok" in r.stdout
    # one group: every body, 2D and 3D, shares one launch table
    env["TLSPH_SERVE_GROUPS"] = "1"
    r = subprocess.run([exe, "6"], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
