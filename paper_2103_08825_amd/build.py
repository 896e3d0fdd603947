"""Builds libstencil.so (every HIP/C++ source under csrc/) for gfx950 with hipcc.

Usage: python -m paper_2103_08825_amd.build [--incremental] [-j N]
Objects go to _build/ at the repository root (not committed); the shared
library is written next to this file, where the binding loads it.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OBJ_DIR = os.path.join(ROOT, "_build", "obj")
GEN_DIR = os.path.join(ROOT, "_build", "gen")  # generated kernel-instance units
LIB = os.path.join(HERE, "libstencil.so")
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=%s" % ARCH,
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I%s" % os.path.join(ROOT, "include"), "-I%s" % CSRC,
    "-Wall", "-Wno-unused-command-line-argument",
]


def _sources():
    sys.path.insert(0, CSRC)
    try:
        import gen_instances
    finally:
        sys.path.pop(0)
    generated = gen_instances.write_units(GEN_DIR)
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")) + generated)


def _headers():
    return (glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(CSRC, "*.inc")) +
            glob.glob(os.path.join(ROOT, "include", "*.h")))


def _deps_newest(dep: str) -> float | None:
    """Newest modification time of the files a make-style dependency file lists
    (None if it is missing or names a file that no longer exists)."""
    try:
        with open(dep) as f:
            text = f.read().replace("\\\n", " ")
    except OSError:
        return None
    _, _, rest = text.partition(":")
    newest = 0.0
    for name in rest.split():
        try:
            newest = max(newest, os.path.getmtime(name))
        except OSError:
            return None
    return newest


def _compile(src: str, incremental: bool, newest_header: float) -> tuple[str, float, str]:
    obj = os.path.join(OBJ_DIR, os.path.basename(src) + ".o")
    dep = obj + ".d"
    if incremental and os.path.exists(obj):
        t = os.path.getmtime(obj)
        deps = _deps_newest(dep)
        newest = deps if deps is not None else max(os.path.getmtime(src), newest_header)
        if t >= newest:
            return obj, 0.0, ""
    t0 = time.time()
    tmp = obj + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-MMD", "-MF", dep, "-c", src, "-o", tmp]
    p = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (p.stdout + p.stderr).splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, msgs))
    os.replace(tmp, obj)
    return obj, time.time() - t0, msgs


def build(incremental: bool = False, jobs: int | None = None, verbose: bool = True) -> str:
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        raise RuntimeError("hipcc not found (%s)" % HIPCC)
    os.makedirs(OBJ_DIR, exist_ok=True)
    srcs = _sources()
    newest = max([os.path.getmtime(h) for h in _headers()] + [0.0])
    jobs = jobs or min(16, os.cpu_count() or 4)
    t0 = time.time()
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {ex.submit(_compile, s, incremental, newest): s for s in srcs}
        for f in cf.as_completed(futs):
            obj, dt, msgs = f.result()
            objs.append(obj)
            if verbose and dt > 0:
                print("  compiled %-28s %6.1fs" % (os.path.basename(futs[f]), dt), flush=True)
                if msgs.strip():
                    print(msgs, flush=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=%s" % ARCH, "-o", tmp] + sorted(objs)
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n%s" % (p.stdout + p.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built %s in %.1fs" % (LIB, time.time() - t0), flush=True)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--incremental", action="store_true")
    ap.add_argument("-j", type=int, default=None)
    a = ap.parse_args(argv)
    build(incremental=a.incremental, jobs=a.j)


if __name__ == "__main__":
    sys.exit(main())
