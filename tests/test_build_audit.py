"""Build audit (CPU): every HIP kernel compiles for gfx950 without scratch
memory (register spills or stack arrays would add HBM traffic the roofline
does not count) and without packed FP32 instructions."""
import os
import re
import subprocess

import pytest

from paper_2211_07260_amd import build as b

# every HIP source of the library (the eight FP32 tile-width units included)
SOURCES = sorted(f for f in os.listdir(b.CSRC) if f.endswith(".hip"))


def test_audit_covers_every_hip_source():
    assert len([s for s in SOURCES if s.startswith("xcorr_f32_tx")]) == 8
    assert {"igemm.hip", "xcorr_f32_batched.hip", "roofline_probe.hip"} <= set(SOURCES)


@pytest.fixture(scope="module")
def device_asm(tmp_path_factory):
    """Device assembly of every source, compiled in parallel."""
    import concurrent.futures as cf
    d = tmp_path_factory.mktemp("asm")

    def one(src):
        out = d / (src + ".s")
        cmd = [b.HIPCC] + [f for f in b.CFLAGS if f != "-fPIC"] + ["--cuda-device-only", "-S",
                                                                   os.path.join(b.CSRC, src), "-o", str(out)]
        subprocess.run(cmd, check=True, capture_output=True)
        return src, out.read_text()

    with cf.ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        return dict(ex.map(one, SOURCES))


@pytest.mark.slow
@pytest.mark.parametrize("src", SOURCES)
def test_no_scratch_no_packed_fp32(src, device_asm):
    asm = device_asm[src]
    sizes = [int(v) for v in re.findall(r"\.private_segment_fixed_size:\s+(\d+)", asm)]
    assert sizes and max(sizes) == 0
    assert not re.search(r"\bv_pk_(fma|mul|add)_f32\b", asm)
