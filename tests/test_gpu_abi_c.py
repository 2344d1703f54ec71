"""The C ABI on its own: tests/native/abi_plane.c (plain C, no Python or
PyTorch in the process) casts a floor seen from 1.7 m against the closed
form t = -o_z / d_z, compares both node formats and the brute-force kernel,
and checks an error path."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu


def test_c_abi_plane():
    exe = os.path.join(ROOT, "tests", "native", "_bin", "abi_plane")
    if not os.path.exists(exe):
        import __graft_entry__
        exe = __graft_entry__.build_abi_driver()
    print(f"running {exe}", flush=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout
