"""Build the HIP library libgkr.so in-tree for gfx950 (hipcc, no JIT).

Usage: python -m paper_2404_10404_amd.build   (or build() from Python)
"""
import concurrent.futures
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgkr.so")
SOURCES = ["gkr_batch_kernel.hip", "gkr_kernels.hip", "gkr_api.hip", "gkr_tuning.cpp", "gkr_verify.cpp",
           "gkr_profile.cpp", "gkr_batch.hip", "gkr_ubench.hip", "gkr_noalloc.hip", "gkr_general.hip", "gkr_gl.hip",
           "gkr_vpd.hip", "gkr_contract.hip"]
# Test helper: the device field-code checker the GPU tests load.
ROOT = os.path.dirname(HERE)
CHECKER_SRC = os.path.join(ROOT, "tests", "native", "fr_device_check.hip")
CHECKER_LIB = os.path.join(ROOT, "tests", "native", "libfrcheck.so")
ARCH = "gfx950"

# Packed fp32 instructions are switched off for every device compilation.
COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _vgpr_spills(remarks: str):
    """(kernel, spilled VGPRs) pairs from the compiler's resource-usage remarks."""
    out, name = [], None
    for line in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"VGPRs Spill: (\d+)", line)
        if m and name:
            out.append((name, int(m.group(1))))
    return out


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    extra = ["-Rpass-analysis=kernel-resource-usage"] if src.endswith(".hip") else []
    cmd = [_hipcc(), "-x", "hip", *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), res.stdout, res.stderr[-6000:]))
    # No kernel may spill vector registers to scratch memory: the persistent
    # batch kernel gave wrong results in stop/resume runs when built with
    # spills, so a build with spills is refused.
    spills = [(k, n) for k, n in _vgpr_spills(res.stderr) if n > 0]
    if spills:
        raise RuntimeError("%s: kernels spill vector registers: %s" % (src, spills))
    return obj


def build_checker() -> str:
    """The device field-code checker of the tests (tests/native/libfrcheck.so)."""
    tmp = CHECKER_LIB + ".tmp"
    cmd = [_hipcc(), "-x", "hip", *COMMON, "-shared", "-o", tmp, CHECKER_SRC]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("checker build failed: %s\n%s" % (" ".join(cmd), res.stderr[-4000:]))
    os.replace(tmp, CHECKER_LIB)
    return CHECKER_LIB


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(9, len(srcs) + 1)) as ex:
        checker = ex.submit(build_checker) if os.path.exists(CHECKER_SRC) else None
        objs = list(ex.map(_compile, srcs))
        if checker is not None:
            checker.result()
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), res.stderr[-4000:]))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
