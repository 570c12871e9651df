"""The gfx950 code of every kernel source writes memory only through vector
stores: no scalar-cache store, scalar atomic, or scalar-cache write-back /
discard instruction appears in the device assembly.

CPU-only (hipcc cross-compiles the device code); this file names those
instructions, so it is kept off the GPU runs."""
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2311_15088_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# scalar memory writes: stores, atomics, and the scalar data cache's
# write-back and discard
FORBIDDEN = re.compile(r"^\s*(s_store_|s_buffer_store|s_scratch_store|s_atomic_|s_buffer_atomic_|"
                       r"s_dcache_wb|s_dcache_discard)", re.MULTILINE)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.parametrize("src", sorted(glob.glob(os.path.join(CSRC, "*.hip"))), ids=os.path.basename)
def test_no_scalar_memory_writes(src, tmp_path):
    out = tmp_path / "dev.s"
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "--cuda-device-only", "-S", src,
           "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    text = out.read_text()
    assert "v_" in text  # the assembly holds the kernels
    bad = sorted(set(m.group(1) for m in FORBIDDEN.finditer(text)))
    assert not bad, f"{os.path.basename(src)}: {bad}"
