"""The search server's host code on the CPU: the worker loop (admission by
budget, retirement, result copies), the batched launch tables and their
graph rebuilds, and the API code they call, built from the library's own
sources against a CPU stand-in of the HIP runtime (tests/host_mock: device
memory is host memory, captured work is replayed in order, the launchers
touch the buffers their kernels would and move the run state as the
kernels do), then driven by a stream of requests that arrive while others
run.  AddressSanitizer with UBSan checks every host access, including
launches that would read freed or stale buffers; ThreadSanitizer checks
the worker against the submitting thread.  No GPU is involved."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
MOCK = os.path.join(HERE, "host_mock")
CSRC = os.path.join(ROOT, "paper_2208_14961_amd", "csrc")
HOST_SOURCES = ["ga_server.hip", "ga_multi.hip", "ga_api.hip", "ga_tuning.hip"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def build(tmp, flags, sources):
    exe = os.path.join(tmp, "served_stream")
    cmd = ["g++", "-std=c++20", "-g", "-O1", *flags, "-I", os.path.join(MOCK, "include"),
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-x", "c++", *sources, "-x", "none",
           os.path.join(MOCK, "mock_rt.cpp"), os.path.join(MOCK, "mock_kernels.cpp"),
           os.path.join(MOCK, "served_stream.cpp"), "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout[-4000:]
    return exe


def run(exe, *args):
    r = subprocess.run([exe, *map(str, args)], stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                       text=True, timeout=600)
    return r.returncode, r.stdout, r.stderr


def test_server_stream_under_address_and_ub_sanitizers(tmp_path):
    exe = build(str(tmp_path), ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                                "-fno-omit-frame-pointer"],
                [os.path.join(CSRC, f) for f in HOST_SOURCES])
    # 2,000 requests, 300 us apart: admissions and retirements interleave
    # with ticks; then 3,000 at once
    for count, gap in ((2000, 300), (3000, 0)):
        rc, out, err = run(exe, count, gap, 5000)
        assert rc == 0 and "all done" in out, (count, gap, out[-2000:], err[-4000:])
        assert "runtime error" not in err, err[-4000:]


def test_server_stream_under_thread_sanitizer(tmp_path):
    # ThreadSanitizer does not intercept the clock-based wait behind
    # condition_variable::wait_for and then misreads the worker's mutex; the
    # build replaces the worker's 20 ms timed wait for new requests by an
    # untimed one (every submission and the stop request notify it)
    src = os.path.join(CSRC, "ga_server.hip")
    with open(src) as f:
        text = f.read()
    timed = "S->cv_work.wait_for(lk, std::chrono::milliseconds(20));"
    assert text.count(timed) == 1
    copy = os.path.join(str(tmp_path), "ga_server.hip")
    with open(copy, "w") as f:
        f.write(text.replace(timed, "S->cv_work.wait(lk);"))
    sources = [copy] + [os.path.join(CSRC, f) for f in HOST_SOURCES[1:]]
    exe = build(str(tmp_path), ["-fsanitize=thread"], sources)
    rc, out, err = run(exe, 1000, 500, 3000)
    assert rc == 0 and "all done" in out, (out[-2000:], err[-4000:])
    assert "WARNING: ThreadSanitizer" not in err, err[-6000:]
