"""Builds libils.so (gfx950) from csrc/ with hipcc.

One translation unit per compiled transform length (generated from
csrc/lengths.def) so the register-DFT instantiations compile in parallel.
Usage:  python -m paper_2003_07504_amd.build [--jobs N] [--incremental]
"""
from __future__ import annotations

import argparse
import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libils.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wno-unused-result"] + DEVICE_FLAGS


# Sources that define the fused ILS pass kernels (device code, launch shapes
# and compiled lengths); the pass counters in profiles/ are valid while these
# are unchanged.
KERNEL_SOURCES = ("fft_reg.hpp", "ils_desc.hpp", "ils_launch.hpp", "ils_passes.hpp", "lengths.def", "ils_persist.hpp",
                  "persist.def")


def source_hash() -> str:
    """Hash of the sources of the fused ILS pass kernels (identifies the
    build that the pass counters were taken on)."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name in KERNEL_SOURCES:
            with open(os.path.join(CSRC, name), "rb") as fh:
                h.update(name.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def lengths():
    out = []
    with open(os.path.join(CSRC, "lengths.def")) as fh:
        for line in fh:
            m = re.match(r"\s*ILS_LEN\((\d+),\s*(\d+),\s*(\d+)\)", line)
            if m:
                out.append(tuple(int(v) for v in m.groups()))
    return out


def persist():
    out = []
    with open(os.path.join(CSRC, "persist.def")) as fh:
        for line in fh:
            m = re.match(r"\s*ILS_PERSIST\(([\d,\s]+)\)", line)
            if m:
                out.append(tuple(int(v) for v in m.group(1).split(",")))
    return out


def _headers_mtime():
    return max(os.path.getmtime(os.path.join(CSRC, f)) for f in os.listdir(CSRC)
               if f.endswith((".hpp", ".h", ".def")))


def _compile(src, obj, incremental, extra=()):
    if incremental and os.path.exists(obj):
        newest = max(os.path.getmtime(src), _headers_mtime())
        # the per-length and persistent kernel units include no public header
        if not os.path.basename(src).startswith(("inst_", "persist_")):
            inc = os.path.join(PKG, "..", "include")
            newest = max([newest] + [os.path.getmtime(os.path.join(inc, h)) for h in os.listdir(inc)])
        if os.path.getmtime(obj) >= newest:
            return obj, ""
    cmd = [HIPCC, *COMMON, *extra, "-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{p.stderr[-4000:]}")
    return obj, p.stderr


def build(jobs: int | None = None, incremental: bool = False, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = []
    for L, P, Q in lengths():
        path = os.path.join(BUILD, f"inst_{L}.hip")
        text = ('#include "../csrc/ils_launch.hpp"\n'
                f"ILS_DEFINE_LEN({L}, {P}, {Q})\n")
        if not os.path.exists(path) or open(path).read() != text:
            with open(path, "w") as fh:
                fh.write(text)
        srcs.append((path, os.path.join(BUILD, f"inst_{L}.o"), ()))
    for spec in persist():
        M, H = spec[0], spec[4]
        path = os.path.join(BUILD, f"persist_{M}_{H}.hip")
        text = ('#include "../csrc/ils_persist.hpp"\n'
                f"ILS_DEFINE_PERSIST({', '.join(str(v) for v in spec)})\n")
        if not os.path.exists(path) or open(path).read() != text:
            with open(path, "w") as fh:
                fh.write(text)
        srcs.append((path, os.path.join(BUILD, f"persist_{M}_{H}.o"), ()))
    srcs.append((os.path.join(CSRC, "ils_api.cpp"), os.path.join(BUILD, "ils_api.o"), ("-x", "hip")))
    for name in sorted(os.listdir(CSRC)):
        if name.endswith(".hip"):
            srcs.append((os.path.join(CSRC, name), os.path.join(BUILD, name[:-4] + ".o"), ()))
    jobs = jobs or min(16, os.cpu_count() or 4)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, s, o, incremental, e) for s, o, e in srcs]
        objs = []
        for f in futs:
            obj, err = f.result()
            objs.append(obj)
            if verbose and err:
                print(err, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"link failed:\n{p.stderr[-4000:]}")
    shutil.move(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--incremental", action="store_true")
    ap.add_argument("--verbose", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.incremental, a.verbose))
