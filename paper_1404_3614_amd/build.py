"""Build libhom.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1404_3614_amd.build

Every .hip source under csrc/ is compiled for gfx950 and linked into one
shared library next to this file.  Packed-FP32 instruction selection is
disabled (-packed-fp32-ops); all float code is scalar or compiler-vectorised
by other means.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhom.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-I", INCLUDE]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def build(verbose=True):
    objs = []
    jobs = []
    for src in sources():
        obj = os.path.join(CSRC, os.path.basename(src)[:-4] + ".o")
        cmd = [HIPCC] + [f for f in FLAGS if f != "-shared"] + ["-c", src, "-o", obj]
        jobs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    ok = True
    for src, p in jobs:
        out, _ = p.communicate()
        if p.returncode != 0:
            ok = False
            sys.stderr.write(out.decode(errors="replace"))
            sys.stderr.write(f"[build] FAILED: {src}\n")
        elif verbose and out.strip():
            txt = "\n".join(l for l in out.decode(errors="replace").splitlines()
                            if "packed-fp32-ops" not in l)
            if txt.strip():
                sys.stderr.write(txt + "\n")
    if not ok:
        raise RuntimeError("hipcc compilation failed")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        sys.stderr.write(r.stdout.decode(errors="replace"))
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    if verbose:
        print(f"[build] {LIB}")
    return LIB


if __name__ == "__main__":
    build()
