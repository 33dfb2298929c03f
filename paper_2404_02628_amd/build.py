"""Builds libpimd.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2404_02628_amd.build   (or call build()).
       python -m paper_2404_02628_amd.build --issue-rates   builds only the stand-alone
       instruction issue-rate program (measure/issue_rates.hip), which is not part of the library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpimd.so")
RATES = os.path.join(HERE, "measure", "issue_rates")   # stand-alone measurement program
SOURCES = ["capi.hip", "k_springs.hip", "k_pair.hip", "k_exchange.hip", "k_integrate.hip", "k_cycle_direct.hip", "k_init.hip", "k_persistent.hip"]
ARCH = os.environ.get("PIMD_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-result",
         # keep the compiler from forming packed-FP32 instructions on its own
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(os.path.dirname(HERE), "include")]


def _compile(src: str, objdir: str) -> str:
    obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(lambda s: _compile(s, objdir), SOURCES))
    tmp = OUT + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libpimd.so failed")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


def build_issue_rates(verbose: bool = False) -> str:
    """The stand-alone issue-rate measurement program (not part of the library)."""
    cmd = ["hipcc", *FLAGS, "-o", RATES, os.path.join(HERE, "measure", "issue_rates.hip")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed on issue_rates.hip")
    if verbose:
        print(f"built {RATES}")
    return RATES


if __name__ == "__main__":
    if "--issue-rates" in sys.argv[1:]:
        build_issue_rates(verbose=True)
    else:
        build(verbose=True)
