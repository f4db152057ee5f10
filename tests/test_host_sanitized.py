"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU): tests/sanitize/build_and_run.py builds a copy of libdg2p whose host
pass is instrumented, and runs the C driver tests/sanitize/abi_host_check.c,
which exercises every entry point's argument, descriptor, parameter and
workspace checks, mesh creation for every dimension, order and boundary kind
(leak detection on).  It caught a signed overflow of the element count
product in dg2p_create_mesh for element counts near 2^31 per axis."""

import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("/opt/rocm/bin/hipcc") is None, reason="needs the ROCm toolchain")
def test_abi_host_checks_under_asan_and_ubsan(tmp_path):
    res = subprocess.run([sys.executable, os.path.join(HERE, "sanitize", "build_and_run.py"), str(tmp_path)],
                         capture_output=True, text=True, timeout=900)
    print(res.stdout[-2000:], res.stderr[-4000:])
    assert res.returncode == 0
    assert "all statuses as expected" in res.stdout
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr
