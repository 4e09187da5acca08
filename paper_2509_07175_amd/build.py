"""Builds libvd.so (all HIP sources, gfx950) in this package directory, and
libvd_probe.so (measured chip peaks for the benchmark's roofline report).

Usage: python -m paper_2509_07175_amd.build  (or build() from Python).
Every kernel is compiled for gfx950 only, with packed FP32 instructions
disabled; host code is part of the same shared library.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvd.so")
PROBE_SRC = os.path.join(HERE, "probe", "peak_probe.hip")
PROBE_LIB = os.path.join(HERE, "libvd_probe.so")
ARCH = os.environ.get("VD_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast", "-Wno-unused-result", "-Wno-unused-value",
]


def build(verbose: bool = False) -> str:
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    objs = []
    procs = []
    for s in srcs:
        o = os.path.join(CSRC, os.path.basename(s)[:-4] + ".o")
        objs.append(o)
        cmd = [hipcc, *FLAGS[:-1], "-c", s, "-o", o]
        cmd = [c for c in cmd if c != "-shared"]
        procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    for s, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out.decode(errors="replace"))
            raise RuntimeError(f"hipcc failed on {os.path.basename(s)}")
        if verbose and out:
            sys.stderr.write(out.decode(errors="replace"))
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        sys.stderr.write(r.stdout.decode(errors="replace"))
        raise RuntimeError("link of libvd.so failed")
    os.replace(tmp, LIB)
    for o in objs:
        try:
            os.remove(o)
        except OSError:
            pass
    cmd = [hipcc, *FLAGS[:-1], PROBE_SRC, "-o", PROBE_LIB + ".tmp"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        sys.stderr.write(r.stdout.decode(errors="replace"))
        raise RuntimeError("build of libvd_probe.so failed")
    os.replace(PROBE_LIB + ".tmp", PROBE_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
