"""The sweeps' index arithmetic (csrc/fv_index.hpp), compiled for the host
with g++ and checked against its plain definition over many grid shapes,
chunk sizes and boundary modes (for the wave strips' lane map: every cell
held once, its stencil in the lanes around it); and the batched launches'
dispatch orders, checked on random tile costs against the properties that
define them (each tile once, one contiguous run per XCD of about equal cost,
costliest first).  No GPU needed."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2104_08571_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
@pytest.mark.parametrize("kmax", [None, 12], ids=["default", "kmax12"])
def test_index_arithmetic(tmp_path, kmax):
    """Built as the library is, and with up to twelve strip tails to a wave
    (the most that fit: tails of one cell)."""
    exe = str(tmp_path / "index_check")
    flags = [] if kmax is None else [f"-DRFV_STRIP_KMAX={kmax}"]
    subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", *flags, "-I", CSRC,
                    os.path.join(ROOT, "tests", "index_check.cpp"), "-o", exe], check=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0 and res.stdout.strip() == "ok", res.stdout + res.stderr
