"""The gfx950 code object built into libfemhip.so: no kernel on the assembly, row,
sort, label-copy or solve path keeps private (scratch) memory.

A local array indexed at run time, or a register spill, puts per-lane data in scratch
memory, and every access to it then goes through the memory pipeline; on the row
passes that cost up to a third of the kernel's time.  The kernel metadata the compiler
writes into the code object records each kernel's private segment size and register
count; this test reads it from the library built here (no kernel is launched).  The
long-row kernels (one workgroup per row of more than 32 / 64 columns, rare) are the
exception and are only reported.
"""
import os
import re
import shutil
import struct
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1804_05156_amd", "libfemhip.so")
LLVM = "/opt/rocm/llvm/bin"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"
TARGET = b"hipv4-amdgcn-amd-amdhsa--gfx950"
HOT = ("k_rows", "k_assemble_2d", "k_assemble_3d", "k_values_to_label", "k_pattern_to_label", "k_label_rows",
       "k_scatter_coords", "k_l1_", "k_l2_bucket", "k_pi", "k_ident", "k_cg_", "k_spmv", "k_batch_pcg",
       "k_grad", "k_upper")
EXEMPT = ("k_assemble_long", "k_rows_long")


def _tool(name):
    p = os.path.join(LLVM, name)
    return p if os.path.exists(p) else shutil.which(name)


def _code_objects(blob):
    """The gfx950 ELF images of every offload bundle in the library's fat binary."""
    out = []
    at = blob.find(MAGIC)
    while at >= 0:
        n = struct.unpack_from("<Q", blob, at + len(MAGIC))[0]
        p = at + len(MAGIC) + 8
        for _ in range(n):
            off, size, tlen = struct.unpack_from("<QQQ", blob, p)
            triple = blob[p + 24:p + 24 + tlen]
            p += 24 + tlen
            if triple == TARGET:
                out.append(blob[at + off:at + off + size])
        at = blob.find(MAGIC, at + 1)
    return out


def _kernels():
    objcopy, readelf = _tool("llvm-objcopy"), _tool("llvm-readelf")
    if not (objcopy and readelf and os.path.exists(LIB)):
        pytest.skip("ROCm LLVM tools or the built library not available")
    with tempfile.TemporaryDirectory() as d:
        fat = os.path.join(d, "fat.bin")
        subprocess.run([objcopy, "--dump-section", f".hip_fatbin={fat}", LIB, os.path.join(d, "lib.so")],
                       check=True, capture_output=True)
        kern = {}
        for j, co in enumerate(_code_objects(open(fat, "rb").read())):
            path = os.path.join(d, f"co{j}.o")
            open(path, "wb").write(co)
            notes = subprocess.run([readelf, "--notes", path], check=True, capture_output=True, text=True).stdout
            for block in notes.split("  - .agpr_count")[1:]:
                name = re.search(r"\.name:\s+(\S+)", block)
                priv = re.search(r"\.private_segment_fixed_size:\s+(\d+)", block)
                vgpr = re.search(r"\.vgpr_count:\s+(\d+)", block)
                if name and priv and vgpr:
                    kern[name.group(1)] = (int(priv.group(1)), int(vgpr.group(1)))
    return kern


def _short(mangled):
    m = re.search(r"(k_[a-z0-9_]+?)(?:I|E)", mangled)
    return m.group(1) if m else mangled


def test_hot_kernels_keep_no_scratch():
    kern = _kernels()
    assert kern, "no gfx950 kernel metadata found in the library"
    hot = {k: v for k, v in kern.items() if _short(k).startswith(HOT) and not _short(k).startswith(EXEMPT)}
    assert len(hot) >= 40, sorted(_short(k) for k in hot)
    for k, (priv, vgpr) in sorted(hot.items()):
        print(f"{_short(k):28s} private {priv:4d} B  VGPRs {vgpr}")
    bad = {_short(k): priv for k, (priv, _) in hot.items() if priv != 0}
    assert not bad, f"kernels with private (scratch) memory: {bad}"
