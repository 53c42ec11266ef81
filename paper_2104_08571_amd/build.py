"""Build libripple_fv.so (HIP, gfx950) in-tree.

Each translation unit is compiled by hipcc to an object, in parallel, and the
objects are linked into paper_2104_08571_amd/libripple_fv.so.  Flags:
  -ffp-contract=off   no implicit fused multiply-add: FMAs appear only where
                      the device code writes them, so every inlined copy of
                      the cell arithmetic rounds identically (bitwise
                      invariance across layouts, tilings, batching and
                      partitioning)
  -packed-fp32-ops    disabled target feature: no packed FP32 instructions
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBRARY = os.path.join(HERE, "libripple_fv.so")
BUILD_DIR = os.path.join(HERE, "_build")
SOURCES = ["fv_kernels.hip", "fv_api.hip", "force2d.hip", "particles.hip"]
ARCH = "gfx950"

HIPCC_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-ffp-contract=off",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wall", "-Wno-unused-result", "-I", INCLUDE, "-I", CSRC]


def _hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    path = os.path.join(rocm, "bin", "hipcc")
    return path if os.path.exists(path) else "hipcc"


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("command failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)
    return res


def build(verbose=False, save_temps=False):
    """Compile and link the library; return its path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    hipcc = _hipcc()
    objs = []
    cmds = []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        cmd = [hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if save_temps:
            cmd += ["-save-temps=obj"]
        cmds.append(cmd)
        objs.append(obj)
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        results = list(ex.map(_run, cmds))
    if verbose:
        for r in results:
            sys.stderr.write(r.stderr)
    tmp = LIBRARY + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIBRARY)
    return LIBRARY


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, save_temps="--save-temps" in sys.argv))
