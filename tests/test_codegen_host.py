"""Properties of the compiled gfx950 kernels, checked on the host from the
assembly hipcc emits for the kernel translation units (no GPU needed):
no kernel spills into accumulation registers or scratch memory, and none
uses packed FP32 arithmetic."""
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2104_08571_amd"))


@pytest.fixture(scope="module", params=["fv_kernels.hip", "force2d.hip", "particles.hip"])
def assembly(request, tmp_path_factory):
    import build
    hipcc = build._hipcc()
    if not (os.path.exists(hipcc) or shutil.which(hipcc)):
        pytest.skip("needs hipcc")
    out = str(tmp_path_factory.mktemp("asm") / (request.param + ".s"))
    cmd = [hipcc, *build.HIPCC_FLAGS, "--cuda-device-only", "-S",
           os.path.join(build.CSRC, request.param), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    with open(out) as f:
        return f.read()


def kernels(asm):
    names = re.findall(r"^(_ZN3rfv\w+):", asm, flags=re.M)
    for n in names:
        start = asm.index(n + ":")
        yield n, asm[start:asm.index(".Lfunc_end", start)]


def test_no_accumulation_register_or_scratch_spills(assembly):
    bad = [n for n, body in kernels(assembly)
           if re.search(r"v_accvgpr_(read|write)|scratch_(load|store)", body)]
    assert not bad, bad
    assert not re.findall(r"\.vgpr_spill_count:\s+[1-9]", assembly)
    assert not re.findall(r"\.private_segment_fixed_size:\s+[1-9]", assembly)


def test_no_packed_fp32(assembly):
    assert not re.search(r"\bv_pk_(fma|mul|add)_f32\b", assembly)
