"""The host code of libgf.so under sanitizers (CPU only, no GPU).

tests/host/harness.cpp drives the host sources (validation, batch planning,
the request engine and its arena allocator, the autotuners, tuning files)
against tests/host/fake_hip.cpp, a stand-in for the HIP runtime and the
kernel launchers.  It is built with ROCm's clang++ as a plain host C++
compiler twice, with AddressSanitizer + UndefinedBehaviorSanitizer and with
ThreadSanitizer (the engine's worker thread, submitters and pollers on
several threads), and any sanitizer report fails the test.  No device code
is built here.  (GCC 11's ThreadSanitizer does not intercept
pthread_cond_clockwait, which libstdc++ uses for timed condition-variable
waits, and then reports the engine's mutex as locked twice; clang's does.)"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1505_00996_amd", "csrc")
HOST = os.path.join(ROOT, "tests", "host")
LIB_SOURCES = ["gf_api.cpp", "gf_ctx.cpp", "gf_tune.cpp", "gf_batch_host.cpp", "gf_engine.cpp"]
SANITIZERS = {
    "asan_ubsan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"],
    "tsan": ["-fsanitize=thread"],
}
ENV = {
    "asan_ubsan": {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0:exitcode=86",
                   "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1:exitcode=87"},
    "tsan": {"TSAN_OPTIONS": "halt_on_error=1:exitcode=88:second_deadlock_stack=1"},
}

CXX = "/opt/rocm/llvm/bin/clang++"
pytestmark = pytest.mark.skipif(not os.path.exists(CXX) or not os.path.isdir("/opt/rocm/include"),
                                reason="needs ROCm's clang++ and the HIP headers")


@pytest.fixture(scope="module")
def binaries(tmp_path_factory):
    out = {}
    d = tmp_path_factory.mktemp("host_sanitizers")
    procs = []
    for kind, flags in SANITIZERS.items():
        exe = str(d / f"harness_{kind}")
        cmd = [CXX, "-std=c++17", "-O1", "-g", *flags, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
               "-I", os.path.join(ROOT, "include"), "-I", CSRC,
               *[os.path.join(CSRC, s) for s in LIB_SOURCES],
               os.path.join(HOST, "fake_hip.cpp"), os.path.join(HOST, "harness.cpp"), "-o", exe, "-lpthread"]
        procs.append((kind, exe, subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True)))
    for kind, exe, pr in procs:
        _, err = pr.communicate(timeout=600)
        assert pr.returncode == 0, f"{kind} build failed:\n{err[-4000:]}"
        out[kind] = exe
    return out


def run(exe, kind, check=""):
    env = dict(os.environ, **ENV[kind])
    pr = subprocess.run([exe] + ([check] if check else []), env=env, capture_output=True, text=True, timeout=600)
    assert pr.returncode == 0 and "host checks passed" in pr.stderr, \
        f"{kind} {check or 'all'}: exit {pr.returncode}\n{pr.stderr[-6000:]}"
    assert "Sanitizer" not in pr.stderr and "runtime error" not in pr.stderr, pr.stderr[-6000:]
    return pr.stderr


def test_asan_ubsan_all_checks(binaries):
    log = run(binaries["asan_ubsan"], "asan_ubsan")
    for name in ("validation", "range", "plan", "tuning", "engine", "calls"):
        assert f"check: {name}" in log


@pytest.mark.parametrize("check", ["engine", "calls", "tuning"])
def test_tsan(binaries, check):
    run(binaries["tsan"], "tsan", check)
