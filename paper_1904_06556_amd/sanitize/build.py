"""Builds and runs host_checks with AddressSanitizer and
UndefinedBehaviorSanitizer on the host code of libvts (device code is built
as usual: each -fsanitize= is given to the host compilation only).

    python -m paper_1904_06556_amd.sanitize.build          # build and run

Objects go to paper_1904_06556_amd/sanitize/_build/.  Leak detection is off
(the HIP runtime keeps allocations until exit); memory errors and undefined
behaviour stop the run with a report.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
sys.path.insert(0, os.path.dirname(PKG))
from paper_1904_06556_amd import build as B  # noqa: E402

OUT_DIR = os.path.join(HERE, "_build")
EXE = os.path.join(OUT_DIR, "host_checks")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
       "-g"]


def _compile(src: str) -> str:
    obj = os.path.join(OUT_DIR, os.path.basename(src) + ".o")
    flags = [f for f in B.FLAGS if f != "-O3"] + ["-O1"]
    cmd = [B.HIPCC, *flags, *SAN, "-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build() -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    srcs = [os.path.join(B.CSRC, s) for s in B.SOURCES] + [os.path.join(HERE, "host_checks.cpp")]
    with cf.ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, srcs))
    cmd = [B.HIPCC, "-pthread", "--offload-arch=gfx950", *SAN, *objs, "-o", EXE]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    return EXE


def run() -> int:
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([EXE], env=env, capture_output=True, text=True)
    sys.stdout.write(r.stdout)
    sys.stderr.write(r.stderr[-4000:])
    return r.returncode


if __name__ == "__main__":
    build()
    sys.exit(run())
