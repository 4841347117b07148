"""The fused solver's code generation for gfx950, read on the CPU from the
built library's own code object (the kernel metadata the compiler records).

The solver kernel is held to 128 VGPRs (4 waves per SIMD); its speed depends on
the column loops fitting that budget, and its HBM traffic on nothing being
spilled to scratch memory (spilled epilogue values once cost 2.2 GB of extra
writes per batched step).  Small source changes have moved the compiler from
no spills to hundreds, inside the loops, so the property is checked on the
metadata of libhsd.so's gfx950 code: every ordinary-grid solver kernel (the
launches the plans make) uses no scratch and at most 128 VGPRs."""

import os
import re
import struct
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1311_4627_amd", "libhsd.so")
LLVM = "/opt/rocm/llvm/bin"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"


def _gfx950_code_objects(fatbin: bytes):
    """The gfx950 entries of the clang offload bundles in a .hip_fatbin section
    (one bundle per linked object: magic, entry count, then per entry its
    offset, size and target id, offsets relative to the bundle)."""
    pos = fatbin.find(MAGIC)
    while pos >= 0:
        n = struct.unpack_from("<Q", fatbin, pos + 24)[0]
        off = pos + 32
        for _ in range(n):
            o, sz, idl = struct.unpack_from("<QQQ", fatbin, off)
            off += 24
            ident = fatbin[off:off + idl].decode()
            off += idl
            if ident.endswith("gfx950") and sz > 0:
                yield fatbin[pos + o:pos + o + sz]
        pos = fatbin.find(MAGIC, pos + 1)


def _kernel_metadata(notes: str):
    lines = notes.split("\n")
    out = {}
    for i, line in enumerate(lines):
        s = line.strip()
        if not (s.startswith(".name:") and "k_solve" in s):
            continue
        fields = {}
        for x in lines[i + 1:i + 60]:
            x = x.strip()
            if x.startswith(".name:") or x.startswith("- .agpr_count"):
                break
            for key in (".private_segment_fixed_size", ".vgpr_count", ".vgpr_spill_count"):
                if x.startswith(key + ":") and key not in fields:
                    fields[key] = int(x.split()[-1])
        out[s.split()[-1]] = fields
    return out


def test_solver_kernels_fit_128_vgprs_without_scratch(tmp_path):
    if not os.path.exists(LIB):
        pytest.skip("libhsd.so is not built")
    if not (os.path.exists(os.path.join(LLVM, "llvm-objcopy")) and os.path.exists(os.path.join(LLVM, "llvm-readelf"))):
        pytest.skip("the ROCm LLVM tools are not available")
    fb = str(tmp_path / "fatbin")
    r = subprocess.run([os.path.join(LLVM, "llvm-objcopy"), f"--dump-section=.hip_fatbin={fb}", LIB,
                        str(tmp_path / "unused.so")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    meta = {}
    for i, co in enumerate(_gfx950_code_objects(open(fb, "rb").read())):
        path = tmp_path / f"co{i}.elf"
        path.write_bytes(co)
        notes = subprocess.run([os.path.join(LLVM, "llvm-readelf"), "--notes", str(path)],
                               capture_output=True, text=True).stdout
        meta.update(_kernel_metadata(notes))
    # template arguments P, R, KG, WAVES, GIVEN, LDSCUM, PERSIST in the mangled name
    pat = re.compile(r"k_solveILi(\d+)ELi(\d+)ELi(\d+)ELi(\d+)ELb([01])ELb([01])ELb([01])E")
    checked = 0
    for name, f in meta.items():
        m = pat.search(name)
        assert m, name
        given, persist = m.group(5) == "1", m.group(7) == "1"
        if given or persist:
            continue
        assert f[".vgpr_count"] <= 128, (name, f)
        assert f[".private_segment_fixed_size"] == 0, (name, f)
        assert f.get(".vgpr_spill_count", 0) == 0, (name, f)
        checked += 1
    # 4 classes (two layouts for classes 0, 1 and 3) x 2 slot-group sizes, launched as ordinary grids
    assert checked == 14, checked
