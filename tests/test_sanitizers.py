"""The library's host code and the oracle under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only, no kernel runs).

* The library built with -fsanitize=address,undefined on its host side
  (`paper_2501_02161_amd.build.build_host_sanitized`) runs the host-path tests
  (tests/test_abi.py: symbol exports, descriptor and mask validation,
  workspace sizing, batch admission checks; tests/test_serving_host.py)
  under clang's ASan runtime.
* The oracle built with the same sanitizers by g++ (`oracle.build(sanitize=True)`)
  runs the oracle's pin, adjoint, heat-generation and level-set tests (all
  but the three largest cases) under gcc's libasan.

Each run is a child process with its runtime preloaded and the sanitized
library selected (LBMADJ_LIB, ORACLE_LIB); it must pass, must have loaded the
sanitized build, and must print no sanitizer report.  UBSan findings abort
(-fno-sanitize-recover), so a report also fails the run.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow

SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
           "OMP_NUM_THREADS": "4"}
REPORTS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")

LOADED = ("import sys; sys.path.insert(0, {root!r}); {load}; "
          "print(sum(l.rstrip().endswith({name!r}) for l in open('/proc/self/maps')) > 0)")


def run(env_extra, args, timeout):
    env = dict(os.environ)
    env.update(SAN_ENV)
    env.update(env_extra)
    r = subprocess.run([sys.executable] + args, cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=timeout)
    out = r.stdout + r.stderr
    return r.returncode, out


def check(env_extra, load, name, tests, timeout):
    rc, out = run(env_extra, ["-c", LOADED.format(root=ROOT, load=load, name=name)], 300)
    assert rc == 0 and out.strip().endswith("True"), f"sanitized {name} was not loaded:\n{out}"
    rc, out = run(env_extra, ["-m", "pytest", "-q", "-x", "-p", "no:cacheprovider"] + tests, timeout)
    tail = "\n".join(out.splitlines()[-30:])
    print(tail, flush=True)
    assert not any(s in out for s in REPORTS), tail
    assert rc == 0, tail


def test_library_host_code_under_asan_ubsan():
    from paper_2501_02161_amd import build
    lib = build.build_host_sanitized()
    check({"LD_PRELOAD": build.asan_runtime(), "LBMADJ_LIB": lib},
          "from paper_2501_02161_amd import lbm; lbm.load_library()", "san/liblbmadj.so",
          ["tests/test_abi.py", "tests/test_serving_host.py"], 900)


def test_oracle_under_asan_ubsan():
    import oracle
    lib = oracle.build(force=True, sanitize=True)
    asan = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    assert os.path.isabs(asan) and os.path.exists(asan), "gcc's libasan.so not found"
    # the real and complex-step forward sweeps, the discrete adjoint, the
    # sensitivity, heat generation, mirror planes, the boundary matrices and
    # the level set on the smaller cases (the largest complex-step cases and
    # the continuous adjoint's long solves are left to the plain run)
    check({"LD_PRELOAD": asan, "ORACLE_LIB": lib}, "import oracle; oracle._load()",
          "liborc_san.so",
          ["tests/test_oracle_pins.py", "tests/test_oracle_adjoint.py",
           "tests/test_oracle_heatgen.py", "tests/test_oracle_levelset.py",
           "-k", "not heat_sink] and not pipe_bend_2d_config and not heatgen_pressure_inlet"],
          1500)
