"""The plain-C consumer of the library (tests/c_abi/check.c, built by
__graft_entry__.build()) run as a child process on the GPU: closed forms of
Eq. (1) for one point, and a status code, through include/cgh.h alone."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def test_c_consumer():
    exe = os.path.join(HERE, "c_abi", "check")
    assert os.path.exists(exe), "tests/c_abi/check is built by __graft_entry__.build()"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr
    assert "c abi ok" in r.stdout
