"""The library's host thread pool (batch planning) on the CPU: compiled with
g++ from its source beside a small driver, loops of many sizes from three
threads at once visit every item exactly once, with the pool on, with one
thread, and off."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1807_07691_amd", "csrc")


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("pool") / "pool_check")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-pthread", "-I", CSRC,
                           os.path.join(ROOT, "tests", "native", "pool_check.cpp"),
                           os.path.join(CSRC, "host_pool.cpp"), "-o", out])
    return out


@pytest.mark.parametrize("threads", ["", "1", "0"])
def test_every_item_once(exe, threads):
    env = dict(os.environ)
    env.pop("GSMAT_HOST_THREADS", None)
    if threads:
        env["GSMAT_HOST_THREADS"] = threads
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "bad 0" in r.stdout and "calls 6000" in r.stdout
