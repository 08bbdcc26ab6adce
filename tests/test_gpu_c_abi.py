"""The library called from plain C (tests/c/abi_consumer.c, built by gcc
against include/dr.h only): a scan reconstructed through the C ABI conserves
intensity, its totals add up and the FP32 and FP64 instances agree.  Needs an
MI355X."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

BIN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "abi_consumer")


def test_plain_c_caller():
    assert os.path.exists(BIN), "tests/c/abi_consumer not built (run the package build)"
    r = subprocess.run([BIN], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("c abi ok"), r.stdout
