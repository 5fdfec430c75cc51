"""Build audit (CPU): every HIP kernel compiles for gfx950 without scratch
memory (register spills or stack arrays would add HBM traffic the roofline
does not count) and without packed FP32 instructions."""
import os
import re
import subprocess

import pytest

from paper_2211_07260_amd import build as b

SOURCES = ["xcorr_f32_tx4.hip", "xcorr_f32_tx8.hip", "xcorr_f32_batched.hip", "igemm.hip",
           "roofline_probe.hip"]


@pytest.mark.slow
@pytest.mark.parametrize("src", SOURCES)
def test_no_scratch_no_packed_fp32(src, tmp_path):
    out = tmp_path / (src + ".s")
    cmd = [b.HIPCC] + [f for f in b.CFLAGS if f != "-fPIC"] + ["--cuda-device-only", "-S",
                                                               os.path.join(b.CSRC, src), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    asm = out.read_text()
    sizes = [int(v) for v in re.findall(r"\.private_segment_fixed_size:\s+(\d+)", asm)]
    assert sizes and max(sizes) == 0
    assert not re.search(r"\bv_pk_(fma|mul|add)_f32\b", asm)
