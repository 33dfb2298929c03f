"""The CPU oracle and the library's host-side planning code under AddressSanitizer and
UndefinedBehaviorSanitizer (leak detection on), built here and run without a GPU.

* The oracle (plain C, gcc): every entry point over 189 small configurations (N = 1..9, P = 2..7,
  d = 1..3, xi in {0, 0.5, 1}, two species, with and without the pair term, thermostatted and
  NVE steps, exact energies, the generator) and its refusals of invalid arguments
  (`tests/native/oracle_sanitize.c`).
* The library (hipcc, sanitizers on the host side only, so the device code is compiled as
  usual): configuration checks, workspace layout and the per-kernel work lists for 2916 plans
  (1 to 300 replicas of uneven N up to 5000, both precisions, d = 1..3, every flag that changes the
  plan, three recursion schedules), invalid configurations, and pimd_create with a missing,
  misaligned or short workspace (`tests/native/plan_sanitize.cpp`).
Any sanitizer report ends the driver with a non-zero status; a planted overflow (one element short
in a buffer) was checked to be reported."""
import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2404_02628_amd", "csrc")
SOURCES = ["capi.hip", "k_springs.hip", "k_pair.hip", "k_exchange.hip", "k_integrate.hip", "k_cycle_direct.hip",
           "k_init.hip", "k_persistent.hip"]
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd[0], r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_san")
        _run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              "-fno-omit-frame-pointer", os.path.join(ROOT, "tests", "native", "oracle_sanitize.c"),
              os.path.join(ROOT, "oracle", "pimd_oracle.c"), "-lm", "-o", exe])
        out = _run([exe])
    assert out.startswith("ok "), out
    assert int(out.split()[1]) == 189


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_plan_code_under_sanitizers():
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", *SAN_HOST,
             "-fno-omit-frame-pointer", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include")]
    with tempfile.TemporaryDirectory() as d:
        def comp(src):
            obj = os.path.join(d, os.path.splitext(os.path.basename(src))[0] + ".o")
            _run(["hipcc", *flags, "-c", src, "-o", obj])
            return obj
        srcs = [os.path.join(CSRC, s) for s in SOURCES] + [os.path.join(ROOT, "tests", "native", "plan_sanitize.cpp")]
        with ThreadPoolExecutor(max_workers=min(len(srcs), os.cpu_count() or 4)) as ex:
            objs = list(ex.map(comp, srcs))
        exe = os.path.join(d, "plan_san")
        _run(["hipcc", "--offload-arch=gfx950", *SAN_HOST, *objs, "-o", exe])
        env = dict(os.environ, UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        out = _run([exe], env=env)
    assert out.startswith("ok "), out
    assert int(out.split()[1]) == 2916
