"""The library's hipcc flags keep packed two-lane FP32 arithmetic out of the
gfx950 device code: a float2 multiply-add kernel compiled with the flags of
build.py contains no packed FP32 add/multiply/FMA instruction, and the same
kernel without the feature flag does (so the check can fail)."""
import os
import re
import shutil
import subprocess

import pytest

from paper_2302_07411_amd import build

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
KERNEL = r"""
#include <hip/hip_runtime.h>
__global__ void k(float2* a, const float2* b, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    float2 x = a[i], y = b[i];
    x.x = x.x * y.x + y.y;
    x.y = x.y * y.y + y.x;
    a[i] = x;
  }
}
"""
PACKED = re.compile(r"\bv_pk_(add|mul|fma)_f32\b")


def _device_asm(tmp_path, flags):
    src = tmp_path / "k.hip"
    src.write_text(KERNEL)
    out = tmp_path / "k.s"
    keep = [f for f in flags if f not in ("-shared", "-fPIC")]
    subprocess.run([HIPCC, *keep, "--cuda-device-only", "-S", str(src), "-o", str(out)],
                   check=True, capture_output=True, text=True)
    return out.read_text()


@pytest.mark.skipif(shutil.which(HIPCC) is None and not os.path.exists(HIPCC), reason="no hipcc")
def test_no_packed_fp32_in_device_code(tmp_path):
    flags = list(build.HIPCC_FLAGS)
    assert not PACKED.search(_device_asm(tmp_path, flags))
    i = flags.index("-packed-fp32-ops")
    without = flags[:i - 3] + flags[i + 1:]
    assert "-packed-fp32-ops" not in without and "-target-feature" not in without
    assert PACKED.search(_device_asm(tmp_path, without))
