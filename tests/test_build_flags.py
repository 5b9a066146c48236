"""The device code carries no packed FP32 arithmetic.

The build hands the device compiler the target-feature flag that turns packed FP32 instructions
off (hipcc's host pass warns that it does not know the feature; the device pass honours it), and
the kernels accumulate their FP32 operator products in FP64. This test reads the gfx950 code
object out of the built library (this repository's own build) and checks that its disassembly
holds no v_pk_*_f32 instruction.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2208_06191_amd import build, mbddc

LLVM = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin")


def _tool(name):
    p = os.path.join(LLVM, name)
    return p if os.path.exists(p) else shutil.which(name)


def test_build_passes_the_flag():
    flags = " ".join(build.HIP_FLAGS)
    assert "-target-feature -Xclang -packed-fp32-ops" in flags


def test_no_packed_fp32_in_device_code(tmp_path):
    objcopy, bundler, objdump = _tool("llvm-objcopy"), _tool("clang-offload-bundler"), _tool("llvm-objdump")
    if not (objcopy and bundler and objdump):
        pytest.skip("LLVM tools of the ROCm install not found")
    if not os.path.exists(mbddc.LIB_PATH):
        pytest.skip("library not built")
    fat, co = tmp_path / "fatbin.bin", tmp_path / "gfx950.co"
    subprocess.run([objcopy, "--dump-section", f".hip_fatbin={fat}", mbddc.LIB_PATH, str(tmp_path / "x.so")],
                   check=True)
    subprocess.run([bundler, "--unbundle", "--type=o", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950",
                    f"--input={fat}", f"--output={co}"], check=True)
    dis = subprocess.run([objdump, "-d", str(co)], check=True, capture_output=True, text=True).stdout
    assert "k_apply_sym" in dis and "v_mfma_f64" in dis      # the kernels are there
    assert "v_mfma_f32_16x16x4" in dis                      # the FP32 factorisation's matrix-core products
    found = sorted(set(re.findall(r"\bv_pk_\w*f32\b", dis)))
    assert not found, found
