"""The one-launch LU sweep protocol (paper_2410_05865_amd/csrc/lu_flow.hpp) on
the CPU: tests/lu_flow_model.cpp runs the header's flow_run on host threads
under ThreadSanitizer (dependencies read with plain loads, so a missing
happens-before edge is a reported race), checks the sweeps' results against a
sequential order, repeated sweeps with the counters reset, and the bounded
wait giving up on a node that never completes.  Two builds with a planted
mistake (completion counts without release; no dependencies at all) must
fail, which shows the check can fail."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lu_flow_model.cpp")
ENV = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")


def _build(tmp_path, define=None):
    exe = str(tmp_path / ("model" if define is None else define))
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread", SRC, "-o", exe]
    if define:
        cmd.insert(1, "-D" + define)
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")


def test_protocol_under_thread_sanitizer(tmp_path):
    exe = _build(tmp_path)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=ENV)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "all ok" in res.stdout
    assert "ok give-up: error word set" in res.stdout
    assert "ThreadSanitizer" not in res.stderr


@pytest.mark.parametrize("define", ["PLANT_RELAXED_SIGNAL", "PLANT_NO_WAITS"])
def test_planted_mistakes_are_caught(tmp_path, define):
    exe = _build(tmp_path, define)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=ENV)
    assert res.returncode != 0
    assert "ThreadSanitizer" in res.stderr or "FAIL" in res.stdout
