"""The C-ABI layer's host logic on the CPU under AddressSanitizer and
UndefinedBehaviorSanitizer (tests/host_harness): api.cpp and registry.cpp are
built with g++ against a host-only stand-in for the HIP runtime, with stub
sweep launchers that track each buffer's time level, together with the
oracle (gcc, same sanitizers).  Covered: argument validation; the pass
choreography of stencil_run (ping-pong order, remainder pass, T = 0, aliased
input and output) for ping-pong and in-place plans; graph recording and
replay, and the fallback to direct launches when capture fails; the autotune
cache key (a plan asking for a depth never receives another plan's) and its
file (written, reloaded in a new process, a corrupt file ignored); the
oracle's entry points on small grids of every dimension."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HH = os.path.join(ROOT, "tests", "host_harness")
CSRC = os.path.join(ROOT, "paper_2103_08825_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not shutil.which("g++") or not os.path.exists("/opt/rocm/include/hip/hip_runtime_api.h"):
        pytest.skip("needs g++ and the HIP headers")
    out = tmp_path_factory.mktemp("host_harness")
    objs = []
    for src in (os.path.join(HH, "harness.cpp"), os.path.join(HH, "hip_stub.cpp"),
                os.path.join(CSRC, "api.cpp"), os.path.join(CSRC, "registry.cpp")):
        obj = str(out / (os.path.basename(src) + ".o"))
        subprocess.run(["g++", "-std=c++17", "-g", "-O1", "-Wall", "-D__HIP_PLATFORM_AMD__",
                        "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include")] + SAN +
                       ["-c", src, "-o", obj], check=True)
        objs.append(obj)
    obj = str(out / "oracle.o")
    subprocess.run(["gcc", "-std=c11", "-g", "-O1", "-fopenmp", "-ffp-contract=off"] + SAN +
                   ["-c", os.path.join(ROOT, "oracle", "oracle.c"), "-o", obj], check=True)
    exe = str(out / "harness")
    subprocess.run(["g++", "-fopenmp"] + SAN + objs + [obj, "-o", exe, "-lm"], check=True)
    return exe, out


def _run(exe, *args, env=None):
    e = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    e.update(env or {})
    p = subprocess.run([exe] + list(args), capture_output=True, text=True, env=e, timeout=120)
    assert p.returncode == 0, p.stdout + p.stderr
    return p.stdout


@pytest.mark.parametrize("scenario", ["validation", "passes", "graph", "oracle"])
def test_host_logic_under_sanitizers(harness, scenario):
    exe, out = harness
    text = _run(exe, scenario, env={"STENCIL_TUNE_CACHE": ""})
    assert "PASS" in text and "FAIL" not in text, text


def test_autotune_cache_file(harness):
    exe, out = harness
    cache = str(out / "tune.txt")
    env = {"STENCIL_TUNE_CACHE": cache}
    _run(exe, "tune", "write", env=env)
    lines = open(cache).read().splitlines()
    assert len(lines) == 2 and all(l.startswith("gfx950 ") for l in lines), lines
    _run(exe, "tune", "load", env=env)        # another process takes the stored choice
    with open(cache, "w") as f:
        f.write("garbage\nsig\tx y z\n")
    _run(exe, "tune", "corrupt", env=env)     # a corrupt file is ignored
