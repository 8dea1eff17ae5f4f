"""Host-side memory safety of the library's C ABI under failing HIP calls.

The host layer (ihdg_api.cpp) is compiled with g++ under AddressSanitizer and
UBSan against a CPU stand-in of the HIP runtime (tests/host_stub) that defers
every asynchronous copy until its stream is synchronised and can make any
runtime call or launch fail.  The harness drives setup, the FP64 / mixed /
GMRES / BiCGStab solve drivers, time stepping and the batch (direct launches
and graph replay) from four threads, failing each of their calls in turn, then
completes the deferred copies.  A host buffer released by the library while a
copy into or out of it is still queued is reported by ASan and fails the test.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
STUB = os.path.join(HERE, "host_stub")
CSRC = os.path.join(ROOT, "paper_1605_03228_amd", "csrc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not available")
    out = str(tmp_path_factory.mktemp("host_stub") / "harness")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-Wno-unused-result", "-I", STUB,
           os.path.join(STUB, "hip_stub.cpp"), os.path.join(STUB, "harness.cpp"),
           os.path.join(CSRC, "ihdg_api.cpp"), os.path.join(CSRC, "ref_tables.cpp"), "-o", out, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def test_every_failing_call_leaves_no_dangling_copy(harness):
    env = dict(os.environ, ASAN_OPTIONS="detect_stack_use_after_return=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([harness, "4"], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:] + "\n" + r.stderr[-6000:])
    assert "bad 0" in r.stdout
    # every scenario ran every failure position on every thread
    assert r.stdout.count("every failure position tried") == 4 * 9


def test_autotuner_times_on_scratch_iterates(harness):
    """The autotuner's timed sweeps ping-pong between two scratch iterates
    per precision, zero both afterwards and never write the iterate a solve
    starts from."""
    r = subprocess.run([harness, "tune"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.stdout[-2000:] + "\n" + r.stderr[-4000:])
    assert "tune ok" in r.stdout
    assert r.stdout.count("on 2 buffers, zeroed 1 1, current iterate untouched 1") == 2
