"""Compiles the device code for gfx950 (hipcc, no GPU needed) and checks every kernel's resource
metadata: no kernel may use scratch memory (a whole-struct select of a 16-byte composite, for
one, is lowered through scratch and made the sample merge rounds of 64-bit pairs twice as
slow), and the hot 32-bit kernels stay within 64 VGPRs, which their occupancy (eight waves per
SIMD) needs."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1002_4464_amd", "csrc")

pytestmark = pytest.mark.slow


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("asm") / "kernels.s")
    subprocess.check_call([hipcc, "-O3", "-std=c++17", "--offload-arch=gfx950",
                           "-munsafe-fp-atomics", "-Xclang", "-target-feature", "-Xclang",
                           "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"),
                           "--cuda-device-only", "-S", os.path.join(CSRC, "kernels.hip"),
                           "-o", out], stderr=subprocess.DEVNULL)
    text = open(out).read()
    text = text[text.index(".amdgpu_metadata"):]
    meta = {}
    for block in re.split(r"\n  - \.", text)[1:]:  # one entry per kernel
        name = re.search(r"\n    \.name:\s+(\S+)", block)
        if not name:
            continue
        fields = dict(re.findall(r"\.(private_segment_fixed_size|vgpr_count|vgpr_spill_count):"
                                 r"\s+(\d+)", block))
        meta[name.group(1)] = {k: int(v) for k, v in fields.items()}
    assert meta, "no kernel metadata found"
    return meta


def test_no_scratch(kernels):
    bad = {k: v for k, v in kernels.items()
           if v.get("private_segment_fixed_size", 0) or v.get("vgpr_spill_count", 0)}
    assert not bad, f"kernels using scratch memory: {bad}"


def test_hot_32bit_kernels_fit_64_vgprs(kernels):
    hot = [k for k in kernels
           if re.search(r"k_tileIjLb0ELi16ELi16384ELi0E|k_gather_bsortIjLb0ELi(2048|4096|6144|8192)E",
                        k)]
    assert hot, "hot kernels not found"
    over = {k: kernels[k]["vgpr_count"] for k in hot if kernels[k]["vgpr_count"] > 64}
    assert not over, f"above 64 VGPRs: {over}"
