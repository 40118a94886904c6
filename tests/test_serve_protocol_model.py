"""The persistent render server's protocol (csrc/serve_protocol.hpp) in a
host-thread model under ThreadSanitizer: a dispatcher thread and worker
threads make the same protocol calls as the kernel's wavefronts, with the
same memory orders, against a host that submits, polls, checks every pixel,
recycles slots and relaunches idle launches (tests/native/serve_protocol_model.cpp).
A race on the plain pixel writes, a tile rendered twice or missed, a request
completed twice or never, or a launch that does not leave fails the test."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_serve_protocol_model_under_tsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not installed")
    exe = str(tmp_path / "serve_protocol_model")
    subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-Wno-tsan", "-D__host__=", "-D__device__=",
                    "-I", os.path.join(ROOT, "paper_2502_01157_amd", "csrc"), "-o", exe,
                    os.path.join(ROOT, "tests", "native", "serve_protocol_model.cpp"), "-pthread"], check=True)
    p = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"))
    out = p.stdout + p.stderr
    assert p.returncode == 0, out[-3000:]
    assert "ThreadSanitizer" not in out, out[-3000:]
    assert "all tiles rendered once" in p.stdout
