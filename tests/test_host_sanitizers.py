"""The network loader under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only): every generated network parses, and deterministic
mutations of the files (truncations, byte changes, dropped or repeated lines,
extreme numbers, stray text) are rejected or accepted without a memory or
undefined-behaviour error.  Each input is passed in a buffer of exactly its
length, so reads past the end are caught."""
import os
import shutil
import subprocess

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2511_10558_amd", "csrc")
ROCM = "/opt/rocm"


@pytest.fixture(scope="module")
def fuzzer(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime.h")):
        pytest.skip("g++ or the ROCm headers are not available")
    out = tmp_path_factory.mktemp("asan") / "parse_fuzz"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", f"-I{CSRC}", f"-I{ROCM}/include", "-D__HIP_PLATFORM_AMD__",
           os.path.join(ROOT, "tests", "host", "parse_fuzz.cpp"), os.path.join(CSRC, "network.cpp"),
           f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib", "-o", str(out)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        pytest.fail("sanitizer build failed:\n" + res.stderr[-3000:])
    return out


def test_network_loader_under_sanitizers(fuzzer, tmp_path):
    files = []
    for name in ("small", "net200", "net500"):
        p = tmp_path / f"{name}.txt"
        synth.write_network(synth.network_for_config(name), p)
        files.append(str(p))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([str(fuzzer), "300", *files], capture_output=True, text=True, env=env, timeout=600)
    report = res.stdout + res.stderr
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
    assert res.returncode == 0, report[-4000:]
    assert res.stdout.count("status 0,") == 3
