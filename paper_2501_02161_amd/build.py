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
OBJ_DIR = os.path.join(HERE, "_build", "obj")
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
        # the kernels' object is kept for the host-sanitized build
        os.makedirs(OBJ_DIR, exist_ok=True)
        os.replace(objs[0], os.path.join(OBJ_DIR, os.path.basename(objs[0])))
    finally:
        for f in objs:
            if os.path.exists(f):
                os.remove(f)
        if os.path.isdir(tmpdir):
            os.rmdir(tmpdir)
    return LIB


SAN_LIB = os.path.join(HERE, "_build", "san", "liblbmadj.so")
# AddressSanitizer + UndefinedBehaviorSanitizer on the host code (each
# -fsanitize= behind -Xarch_host; device code is never instrumented).  The host
# sources (lbm_host.hip, lbm_batch.hip: descriptor and mask validation,
# workspace sizing, batch admission and scheduling) are compiled with them; the
# kernels' source, whose host side is only launch wrappers, is linked as the
# plain build compiled it.  The host paths run without a GPU; load the library
# with clang's ASan runtime preloaded (asan_runtime()).
SAN_FLAGS = ["-std=c++17", "-O1", "-g", f"--offload-arch={ARCH}", "-fPIC", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined",
             "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include")]


def asan_runtime() -> str:
    """Path of the clang ASan runtime the sanitized host library needs."""
    r = subprocess.run([hipcc(), "--print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("clang's libclang_rt.asan-x86_64.so not found")
    return path


def build_host_sanitized(verbose: bool = False) -> str:
    """Build SAN_LIB: the host sources with ASan + UBSan, linked with the
    kernels' object of the plain build (rebuilt first if it is missing or
    older than its sources)."""
    kobj = os.path.join(OBJ_DIR, os.path.basename(SOURCES[0]) + ".o")
    newest = max(os.path.getmtime(f) for f in [SOURCES[0]] + HEADERS)
    if not os.path.exists(kobj) or os.path.getmtime(kobj) < newest:
        build(verbose)
    sdir = os.path.dirname(SAN_LIB)
    os.makedirs(sdir, exist_ok=True)
    objs = [os.path.join(sdir, os.path.basename(s) + f".{os.getpid()}.o") for s in SOURCES[1:]]
    procs = []
    for src, obj in zip(SOURCES[1:], objs):
        cmd = [hipcc()] + SAN_FLAGS + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
    try:
        if any(pr.wait() != 0 for pr in procs):
            raise RuntimeError("hipcc failed compiling the sanitized library")
        tmp = SAN_LIB + f".tmp{os.getpid()}"
        link = [hipcc(), f"--offload-arch={ARCH}", "-fPIC", "-shared", "-Xarch_host",
                "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan",
                "-o", tmp, kobj] + objs
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
        os.replace(tmp, SAN_LIB)
    finally:
        for f in objs:
            if os.path.exists(f):
                os.remove(f)
    return SAN_LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_host_sanitized(verbose=True))
    else:
        print(build(verbose=True))
