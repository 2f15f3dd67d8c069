"""Build libpicount.so (gfx950) from the HIP sources in csrc/ with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libpicount.so")
SOURCES = ["pc_tables.hip", "pc_leaves.hip", "pc_sieve.hip", "pc_plan.hip", "pc_batch.hip", "pc_seed.hip", "pc_host.hip"]
ARCH = os.environ.get("PICOUNT_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = ["hipcc", *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


# The GPU tests' device libraries (tests/device): each a shared library of its
# own, compiled from the test's source against csrc/pc_device.h: the check of
# the device quotient helpers, the comparison of two pi tables, and the
# micro-benchmarks of the GPU's peaks.
DEVICE_TESTS = [(os.path.join(ROOT, "tests", "device", src), os.path.join(ROOT, "tests", "device", lib))
                for src, lib in (("div_check.hip", "libdivcheck.so"),
                                 ("pi_table_bench.hip", "libpitable.so"),
                                 ("peaks.hip", "libpeaks.so"))]


def _device_test(src: str, lib: str) -> str:
    tmp = lib + ".tmp"
    cmd = ["hipcc", *FLAGS, "-shared", src, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES) + len(DEVICE_TESTS)) as ex:
        devs = [ex.submit(_device_test, src, lib) for src, lib in DEVICE_TESTS
                if os.path.exists(src)]
        objs = list(ex.map(_compile, SOURCES))
        for d in devs:
            d.result()
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
