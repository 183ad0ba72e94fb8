"""Register budgets of the built kernels, read from the gfx950 code-object metadata inside libsmcgw.so (no GPU).

The persistent NUTS kernel runs one particle per slot of four wavefronts; three slots per CU need at most
168 VGPRs per lane (512 / 3, in steps of 8).  An out-of-line tree step shared with another kernel takes the
loosest register budget of its callers, so a new caller with a looser launch bound can silently cost a slot per
CU: this test fails then.
"""
import os
import re
import struct
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2601_02336_amd", "lib", "libsmcgw.so")
READELF = "/opt/rocm/llvm/bin/llvm-readelf"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"


def _code_objects(blob: bytes):
    """Every gfx950 code object of the offload bundles stored in the library."""
    out, pos = [], blob.find(MAGIC)
    while pos >= 0:
        p = pos + len(MAGIC)
        (n,) = struct.unpack_from("<Q", blob, p)
        p += 8
        for _ in range(n):
            off, size, tlen = struct.unpack_from("<QQQ", blob, p)
            p += 24
            triple = blob[p:p + tlen].decode()
            p += tlen
            if "gfx950" in triple and size > 0:
                out.append(blob[pos + off:pos + off + size])
        pos = blob.find(MAGIC, pos + 1)
    return out


def _kernel_metadata():
    if not os.path.exists(LIB) or not os.path.exists(READELF):
        pytest.skip("needs the built library and llvm-readelf")
    with open(LIB, "rb") as f:
        blob = f.read()
    kernels = {}
    for co in _code_objects(blob):
        with tempfile.NamedTemporaryFile(suffix=".co") as t:
            t.write(co)
            t.flush()
            notes = subprocess.run([READELF, "--notes", t.name], capture_output=True, text=True, check=True).stdout
        for block in notes.split("  - .agpr_count:")[1:]:
            name = re.search(r"\.name:\s+(\S+)", block)
            vgpr = re.search(r"\.vgpr_count:\s+(\d+)", block)
            if name and vgpr:
                kernels[name.group(1)] = {
                    "vgpr": int(vgpr.group(1)),
                    "vgpr_spill": int(re.search(r"\.vgpr_spill_count:\s+(\d+)", block).group(1)),
                    "scratch": int(re.search(r"\.private_segment_fixed_size:\s+(\d+)", block).group(1)),
                }
    return kernels


def test_nuts_kernel_keeps_three_slots_per_cu():
    k = _kernel_metadata()
    nuts = {n: v for n, v in k.items() if n.startswith("_ZN5smcgw11nuts_kernelILi") and "ELi4EEEv" in n}
    assert nuts, "no 4-wavefront NUTS kernel found in the library"
    for n, v in sorted(nuts.items()):
        print(f"{n[:48]}: {v}")
        assert v["vgpr"] <= 168, n
    # the batched likelihood's bin loop runs without spills
    bins = {n: v for n, v in k.items() if "bins_mixed_kernel" in n}
    assert bins and all(v["vgpr_spill"] == 0 and v["scratch"] == 0 for v in bins.values())
