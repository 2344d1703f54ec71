"""Host-side sanitizers over the request server (mock device, no GPU).

librcast is rebuilt with ThreadSanitizer, then with AddressSanitizer +
UndefinedBehaviorSanitizer, on host code only (device code is compiled as
usual and never runs: the mock context makes no HIP call), and a
multi-threaded C++ stress driver (tests/native/serve_stress.cpp) runs
against each build.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2509_17390_amd", "csrc")
from paper_2509_17390_amd.build import SOURCES  # every source of the library
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

pytestmark = pytest.mark.timeout(600)


def _build_and_run(tmp, san_flags, env_extra):
    common = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17",
              "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(tmp, src + ".o")
        objs.append(obj)
        procs.append(subprocess.Popen([HIPCC, *common, *san_flags, "-c",
                                       os.path.join(CSRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out.decode()[-3000:]
    drv = os.path.join(tmp, "serve_stress.o")
    r = subprocess.run([HIPCC, *common, *san_flags, "-c", "-o", drv,
                        os.path.join(ROOT, "tests", "native", "serve_stress.cpp")],
                       capture_output=True, text=True)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    exe = os.path.join(tmp, "serve_stress")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", *san_flags, "-o", exe, drv, *objs],
                       capture_output=True, text=True)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "serve_stress: ok" in r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_serve_threadsanitizer():
    with tempfile.TemporaryDirectory() as tmp:
        _build_and_run(tmp, ["-Xarch_host", "-fsanitize=thread"],
                       {"TSAN_OPTIONS": "halt_on_error=1 second_deadlock_stack=1"})


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_serve_address_and_ub_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        _build_and_run(tmp, ["-Xarch_host", "-fsanitize=address", "-Xarch_host",
                             "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all"],
                       {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0",
                        "UBSAN_OPTIONS": "print_stacktrace=1"})
