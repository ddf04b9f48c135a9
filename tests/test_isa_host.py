"""The gfx950 code of every kernel, compiled here from source, writes memory
through vector instructions only: no scalar-cache stores or atomics (and no
scalar-cache write-back or discard)."""
import os
import re
import subprocess
import tempfile

import pytest

from paper_2510_03312_amd import build as hip_build

SCALAR_WRITE = re.compile(r"^\s+s_(store|atomic|buffer_store|buffer_atomic|dcache_wb|dcache_discard)\w*",
                          re.M)


@pytest.mark.skipif(not os.path.exists(hip_build.HIPCC), reason="hipcc not available")
@pytest.mark.parametrize("src", hip_build.SOURCES)
def test_no_scalar_memory_writes(src):
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "k.s")
        flags = [f for f in hip_build.FLAGS if f != "-fPIC"]
        subprocess.run([hip_build.HIPCC, *flags, "--cuda-device-only", "-S",
                        os.path.join(hip_build.CSRC, src), "-o", out], check=True,
                       capture_output=True)
        asm = open(out).read()
    assert "s_endpgm" in asm
    hits = SCALAR_WRITE.findall(asm)
    assert not hits, hits[:5]
