"""libacs's host sources built with the address and undefined-behaviour
sanitizers, against a host stand-in of the HIP runtime (tests/hostsan), and
driven through the graph-per-input RL loop, graph recording and replay, the
in-order, plain, events and manual paths, the RL drivers waiting for each
step's island plan on the host-side paths, and submissions with hundreds of
ranges.  Any sanitizer report, leak (other than the graph module's
process-lifetime stream pool) or misuse of a runtime object (a destroyed
stream, event or graph used again) fails the test.  CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "hostsan")
CSRC = os.path.join(ROOT, "paper_2401_12377_amd", "csrc")
HOST_SOURCES = ["window.cpp", "paths.cpp", "device_path.cpp", "abi.cpp", "workloads.cpp", "graph.cpp", "serve.cpp"]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("hostsan") / "driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__",
           "-I", SAN, "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    cmd += [os.path.join(CSRC, s) for s in HOST_SOURCES]
    cmd += [os.path.join(SAN, "fake_hip.cpp"), os.path.join(SAN, "driver.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


@pytest.mark.parametrize("part", ["graphs", "replay", "paths", "ranges", "rlrun"])
def test_host_code_under_sanitizers(driver, part):
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               LSAN_OPTIONS=f"suppressions={os.path.join(SAN, 'lsan.supp')}:print_suppressions=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([driver, part], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert r.stdout.strip().endswith("ok")
    alive = [l for l in r.stdout.splitlines() if l.startswith("alive:")][0].split()
    counts = dict(zip(alive[1::2], map(int, alive[2::2])))
    # nothing left behind but the graph module's reusable launch stream(s)
    assert counts["events"] == counts["graphs"] == counts["execs"] == counts["device"] == counts["host"] == 0
    assert counts["streams"] <= 1
