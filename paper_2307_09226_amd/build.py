"""Build librs.so (gfx950 HIP kernels + C ABI) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "librs.so")
SOURCES = ["rs_api.hip", "rs_plain.hip", "rs_mfma.hip", "rs_reduce.hip", "rs_session.hip", "rs_rd.hip",
           "rs_scene.hip", "rs_nufft.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # the binary64 recipe must round exactly as written
    "-ffp-contract=off",
    # no packed fp32 arithmetic in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("command failed: " + " ".join(cmd) + "\n" + res.stdout + res.stderr)
    return res


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every HIP source for gfx950 and link librs.so; returns its path."""
    with tempfile.TemporaryDirectory(prefix="rs_build_") as tmp:
        objs = []

        def compile_one(src):
            obj = os.path.join(tmp, src + ".o")
            _run([HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
            return obj

        with ThreadPoolExecutor(max_workers=max(1, min(jobs, len(SOURCES)))) as ex:
            objs = list(ex.map(compile_one, SOURCES))
        out_tmp = LIB + ".tmp"
        _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", out_tmp,
              "-lpthread"])
        os.replace(out_tmp, LIB)
    if verbose:
        print("built", LIB, file=sys.stderr)
    return LIB


TEST_PRIMS_SRC = os.path.join(ROOT, "tests", "csrc", "rs_prims.hip")
TEST_PRIMS_LIB = os.path.join(ROOT, "tests", "csrc", "librs_prims.so")


def build_test_prims(verbose: bool = False) -> str:
    """Compile the test-only primitive library (tests/csrc) with the
    library's own flags; returns its path."""
    out_tmp = TEST_PRIMS_LIB + ".tmp"
    _run([HIPCC, *FLAGS, "-shared", TEST_PRIMS_SRC, "-o", out_tmp])
    os.replace(out_tmp, TEST_PRIMS_LIB)
    if verbose:
        print("built", TEST_PRIMS_LIB, file=sys.stderr)
    return TEST_PRIMS_LIB


def device_asm(src: str) -> str:
    """Device assembly of one source (for inspection of the generated code)."""
    with tempfile.TemporaryDirectory(prefix="rs_asm_") as tmp:
        out = os.path.join(tmp, "k.s")
        _run([HIPCC, *FLAGS, "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out])
        return open(out).read()


if __name__ == "__main__":
    build(verbose=True)
