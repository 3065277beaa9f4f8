"""Build the gfx950 shared library ``_build/liblbmadj.so`` with hipcc.

Run ``python -m paper_2501_02161_amd.build`` (or ``__graft_entry__.build()``).
hipcc cross-compiles for gfx950 without a GPU present.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", n) for n in ("lbm_kernels.hip", "lbm_host.hip", "lbm_batch.hip")]
HEADERS = [os.path.join(ROOT, "include", "lbmadj.h"), os.path.join(HERE, "csrc", "lbm_internal.h")]
LIB = os.path.join(HERE, "_build", "liblbmadj.so")
ARCH = os.environ.get("LBMADJ_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


FLAGS = ["-std=c++17", "-O3", f"--offload-arch={ARCH}", "-fPIC",
         # packed-FP32 instructions stay off: the compiler may not emit v_pk_*_f32
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
         "-I", os.path.join(ROOT, "include")]


def compile_commands(tmpdir: str) -> list:
    """One hipcc -c per source (run in parallel), then the shared-library link."""
    objs = [os.path.join(tmpdir, os.path.basename(src) + ".o") for src in SOURCES]
    cc = [[hipcc()] + FLAGS + ["-c", src, "-o", obj] for src, obj in zip(SOURCES, objs)]
    return cc, objs


def build(verbose: bool = False) -> str:
    """Compile the library (always) and return its path."""
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    tmpdir = os.path.join(os.path.dirname(LIB), f"obj{os.getpid()}")
    os.makedirs(tmpdir, exist_ok=True)
    tmp = LIB + f".tmp{os.getpid()}"
    cc, objs = compile_commands(tmpdir)
    link = [hipcc(), f"--offload-arch={ARCH}", "-fPIC", "-shared", "-o", tmp] + objs
    try:
        procs = []
        for cmd in cc:
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                          text=True))
        failed = False
        for pr in procs:
            out, _ = pr.communicate()
            if pr.returncode != 0:
                sys.stderr.write(out)
                failed = True
        if failed:
            raise RuntimeError("hipcc failed compiling liblbmadj.so")
        if verbose:
            print(" ".join(link), flush=True)
        r = subprocess.run(link, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed linking liblbmadj.so")
        os.replace(tmp, LIB)
    finally:
        for f in objs:
            if os.path.exists(f):
                os.remove(f)
        if os.path.isdir(tmpdir):
            os.rmdir(tmpdir)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
