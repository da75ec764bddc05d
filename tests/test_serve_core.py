"""The serving scheduler (paper_2501_05520_amd/csrc/serve_core.h) on the CPU with
a sleeping test double as executor, built with g++ under ThreadSanitizer and
under AddressSanitizer: admission by memory, batching limits, deadlines, drain
on shutdown, 32 client threads."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "native", "serve_core_test.cpp")


@pytest.mark.parametrize("sanitizer", ["thread", "address"])
def test_serve_core(tmp_path, sanitizer):
    exe = tmp_path / f"serve_core_{sanitizer}"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-pthread", f"-fsanitize={sanitizer}", SRC, "-o", str(exe)],
                   check=True)
    env = dict(os.environ)
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "WARNING: ThreadSanitizer" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert "all checks passed" in r.stdout
