"""Builds the HIP library ``libtlsph_dr.so`` for gfx950 with hipcc.

The setup translation unit (cell binning, neighbour search) is compiled with -ffp-contract=off so
that the neighbour lists and colours round exactly as IEEE double arithmetic written out
operation by operation.  Every translation unit disables packed FP32 instructions.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libtlsph_dr.so")
SOURCES = ["setup.hip", "step.hip", "damp.hip", "api.hip", "serve.hip"]
ARCH = os.environ.get("TLSPH_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-Wall", "-Wno-unused-function", f"-I{INCLUDE}", f"-I{CSRC}"]
PER_FILE = {"setup.hip": ["-ffp-contract=off"]}


def hipcc() -> str:
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(verbose: bool = False, jobs: int = 4, defines=(), out: str = LIB, objdir: str = None) -> str:
    """Compile every source and link the shared library (always rebuilds).  ``defines`` are extra
    -D tuning constants (see the TLSPH_* macros in csrc/)."""
    objdir = objdir or os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [hipcc(), "-c", *COMMON, *[f"-D{d}" for d in defines], *PER_FILE.get(src, []), os.path.join(CSRC, src),
               "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        while len([p for _, p in procs if p.poll() is None]) >= jobs:
            procs[0][1].wait()
    failed = []
    for src, p in procs:
        msg = p.communicate()[0].decode(errors="replace")
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write(msg)
        elif verbose and msg.strip():
            sys.stderr.write(msg)
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    fd, tmp = tempfile.mkstemp(prefix="libtlsph_dr.", suffix=".so", dir=os.path.dirname(out))
    os.close(fd)
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-Wl,--no-undefined", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
