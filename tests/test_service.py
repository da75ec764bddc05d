"""The socket front end (paper_2501_05520_amd/csrc/service_core.h) on the CPU: a
C++ test program built with g++ under ThreadSanitizer and AddressSanitizer (16 client
connections, requests of random sizes including empty ones, protocol errors,
shutdown with an open connection) and the Python client of trk.py against the
same service in serve mode."""
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "native", "service_test.cpp")


def _build(tmp_path, sanitizer):
    exe = tmp_path / f"service_{sanitizer}"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-pthread", f"-fsanitize={sanitizer}", SRC, "-o", str(exe)],
                   check=True)
    env = dict(os.environ)
    env.pop("LD_PRELOAD", None)
    return exe, env


@pytest.mark.parametrize("sanitizer", ["thread", "address"])
def test_service_core(tmp_path, sanitizer):
    exe, env = _build(tmp_path, sanitizer)
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "WARNING: ThreadSanitizer" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert "all checks passed" in r.stdout


def test_python_client(tmp_path):
    from paper_2501_05520_amd.trk import ServiceClient
    exe, env = _build(tmp_path, "address")
    p = subprocess.Popen([str(exe), "--serve"], stdin=subprocess.PIPE, stdout=subprocess.PIPE,
                         stderr=subprocess.PIPE, text=True, env=env)
    try:
        port = int(p.stdout.readline())
        cl = ServiceClient("127.0.0.1", port)
        rng = np.random.default_rng(0)
        for n in (0, 1, 37, 999):
            x = np.zeros((n, 3), np.float32)
            x[:, 0] = rng.integers(0, 100000, n)
            status, labels, info, lat = cl.request(x)
            assert status == 0 and info["n_hits"] == n and lat >= 0
            assert np.array_equal(labels, x[:, 0].astype(np.int32))
        status, labels, _, _ = cl.request(np.zeros((5000, 3), np.float32))   # beyond the service's max_hits
        assert status == -1 and labels is None
        cl.close()
    finally:
        p.stdin.close()
        p.wait(timeout=30)
    assert p.returncode == 0, p.stderr.read()
    assert "ERROR: AddressSanitizer" not in p.stderr.read()
