"""Build the gfx950 HIP library ``libcdm.so`` in-tree with hipcc.

Every kernel source under ``csrc/`` is compiled for gfx950 only.  Packed FP32
instructions are disabled for all device code (``-packed-fp32-ops``).
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libcdm.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", INCLUDE, "-I", CSRC]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


# host pass only: AddressSanitizer and UndefinedBehaviorSanitizer for the library's CPU
# code (descriptor validation, planning); the device code is built as always
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all",
                 "-Xarch_host", "-fno-omit-frame-pointer"]
HOST_SANITIZE_LINK = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-shared-libsan"]


def build(verbose: bool = False, jobs: int = 8, host_sanitize: bool = False, out: str | None = None) -> str:
    """Compile every source to an object (in parallel) and link libcdm.so (or `out`).
    host_sanitize: the host-sanitizer build (objects kept apart from the plain ones)."""
    objdir = os.path.join(PKG, "_build_san" if host_sanitize else "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [HIPCC] + FLAGS + (HOST_SANITIZE if host_sanitize else []) + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _drain(procs)
    _drain(procs)
    lib = out or LIB
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + (HOST_SANITIZE_LINK if host_sanitize else []) + \
        ["-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


def _drain(procs):
    failed = []
    while procs:
        src, p = procs.pop(0)
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if p.returncode != 0:
            failed.append((src, "\n".join(lines)))
        elif lines:
            sys.stderr.write("\n".join(lines) + "\n")
    if failed:
        msg = "\n".join("%s:\n%s" % f for f in failed)
        raise RuntimeError("hipcc failed:\n" + msg)


if __name__ == "__main__":
    print(build(verbose=True))
