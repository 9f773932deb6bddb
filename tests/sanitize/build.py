"""Build _build/asan/host_checks: the host-only code (oracle, input
generator, libagg's host code) with AddressSanitizer and
UndefinedBehaviorSanitizer, linked with tests/sanitize/host_checks.cpp.

The sanitizers instrument host code only: every hipcc line passes them with
-Xarch_host, so the device code is built as usual.  Objects are rebuilt when
a source is newer than the binary.

    python tests/sanitize/build.py
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2606_10030_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(ROOT, "_build", "asan")
BIN = os.path.join(OUT, "host_checks")
ROCM = "/opt/rocm"
CLANG = os.path.join(ROCM, "llvm", "bin", "clang")
CLANGXX = os.path.join(ROCM, "llvm", "bin", "clang++")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
HIP_SOURCES = ["agg_kernels.hip", "agg_api.hip", "agg_tuner.hip", "agg_serve.hip", "agg_pack.hip",
               "agg_filter.hip", "agg_groupby.hip"]
C_SOURCES = [os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "datagen", "datagen.c")]


def _commands():
    cmds = []
    for src in C_SOURCES:
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        cmds.append((src, obj, [CLANG, "-O1", "-g", "-std=gnu11", "-ffp-contract=off", *SAN, "-c", src, "-o", obj]))
    for name in HIP_SOURCES:
        src = os.path.join(CSRC, name)
        obj = os.path.join(OUT, name + ".o")
        cmds.append((src, obj, [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-ffp-contract=off",
                                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                                "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                                "-Xarch_host", "-fno-sanitize-recover=undefined",
                                "-Xarch_host", "-fno-omit-frame-pointer",
                                "-I", INCLUDE, "-I", CSRC, "-c", src, "-o", obj]))
    drv = os.path.join(HERE, "host_checks.cpp")
    cmds.append((drv, os.path.join(OUT, "host_checks.o"),
                 [CLANGXX, "-O1", "-g", "-std=c++17", *SAN, "-I", INCLUDE, "-c", drv, "-o",
                  os.path.join(OUT, "host_checks.o")]))
    return cmds


def _stale(src, obj, extra):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(p) > t for p in [src, *extra])


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    headers = [os.path.join(INCLUDE, "agg.h")] + [os.path.join(CSRC, f) for f in os.listdir(CSRC)
                                                   if f.endswith(".hpp")]
    todo = [c for c in _commands() if _stale(c[0], c[1], headers)]

    def run(cmd):
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"failed: {' '.join(cmd)}\n{r.stderr[-4000:]}")

    jobs = max(1, min(len(todo), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(run, c[2]) for c in todo]:
            f.result()
    objs = [c[1] for c in _commands()]
    if todo or not os.path.exists(BIN):
        run([CLANGXX, *SAN, *objs, "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lpthread",
             "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", BIN])
    return BIN


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
