"""Build the gfx950 shared library libqmc.so in-tree with hipcc.

Every source under csrc/ is compiled for gfx950 only.  Packed FP32 vector
instructions are switched off for all device code, and code objects use
version 5 so that the HIP runtime bundled with PyTorch can load them.
"""

from __future__ import annotations

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libqmc.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    "--offload-arch=gfx950",
    "-mcode-object-version=5",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + INCLUDE,
    "-I" + CSRC,
    "-Wall",
    "-Wno-unused-function",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _embed_device_source(gendir: str) -> None:
    """qmc_device.h as a C++ raw string literal, compiled into the library so
    the run-time specialiser can hand it to hiprtc."""
    src = open(os.path.join(CSRC, "qmc_device.h")).read()
    assert ")QMCSRC\"" not in src
    out = os.path.join(gendir, "qmc_device_src.inc")
    text = 'R"QMCSRC(' + src + ')QMCSRC"\n'
    if not os.path.exists(out) or open(out).read() != text:
        with open(out, "w") as fh:
            fh.write(text)


def build(verbose: bool = False, jobs: int = 8) -> str:
    objdir = os.path.join(ROOT, "_build", "obj")
    gendir = os.path.join(ROOT, "_build", "gen")
    os.makedirs(objdir, exist_ok=True)
    os.makedirs(gendir, exist_ok=True)
    _embed_device_source(gendir)
    procs = []
    objs = []
    t0 = time.time()
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        lang = ["-x", "hip"]
        cmd = [HIPCC] + COMMON + ["-I" + gendir] + lang + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        while sum(p.poll() is None for _, p in procs) >= jobs:
            time.sleep(0.05)
    failed = False
    for src, p in procs:
        out = p.communicate()[0].decode()
        if p.returncode != 0:
            failed = True
            sys.stderr.write(f"--- {os.path.basename(src)}\n{out}\n")
        elif verbose and out.strip():
            sys.stderr.write(out)
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lhiprtc", "-lpthread"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s", flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
