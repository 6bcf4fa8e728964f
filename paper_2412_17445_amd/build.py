"""Build the HIP shared library libpff.so for gfx950 (in-tree)."""

from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpff.so")
SOURCES = [os.path.join(HERE, "csrc", "pff.hip"), os.path.join(HERE, "csrc", "server.hip")]
HEADERS = [os.path.join(HERE, "csrc", f) for f in
           ("common.hpp", "fastdiv.hpp", "fft.hpp", "pointlaw.hpp", "passes.hpp", "pipes.hpp",
            "krylov.hpp", "batch.hpp")]
HEADERS.append(os.path.join(ROOT, "include", "pff.h"))


def hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags(arch="gfx950"):
    return ["-O3", "-std=c++17", f"--offload-arch={arch}", "-fPIC",
            # packed FP32 instructions are kept out of the device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include")]


def command(out=LIB, arch="gfx950", extra=()):
    return [hipcc(), *flags(arch), "-shared", "-o", out, *SOURCES, *extra]


def build(verbose=False):
    """Compile libpff.so (always recompiles; writes atomically).  The sources
    compile in parallel to objects, then link."""
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(HERE, "_build", os.path.basename(src) + ".o")
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        cmd = [hipcc(), *flags(), "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
        objs.append(obj)
    errs = []
    for p in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            errs.append(out + err)
    if errs:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *flags(), "-shared", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError("hipcc link failed:\n" + proc.stdout + proc.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
