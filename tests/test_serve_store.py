"""Host logic of the serving loop (no GPU): the request store stays bounded
over a long run, results survive until released, and a failed scratch
reservation defers a query without dropping or reordering it.  The C++ test
driver is built with g++ (AddressSanitizer and UndefinedBehaviorSanitizer
on) against the library's own header and run."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_serve_store(tmp_path):
    exe = str(tmp_path / "serve_store_test")
    src = os.path.join(ROOT, "tests", "cpp", "serve_store_test.cpp")
    inc = os.path.join(ROOT, "paper_2509_24815_amd", "csrc")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-Wall", "-Wextra", "-Werror", "-fsanitize=address,undefined",
           "-I", inc, src, "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True)
    if b.returncode != 0:
        pytest.fail(b.stderr[-2000:])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "serve store ok" in r.stdout
