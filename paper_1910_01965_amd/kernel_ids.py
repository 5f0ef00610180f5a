"""Identity of the library's device kernels, for counter records.

A rocprofv3 counter reading (HBM bytes or VALU instructions per dispatch)
describes one build of one kernel.  The id of a kernel is the first 16 hex
digits of the SHA-256 of its gfx950 machine code followed by its 64-byte
kernel descriptor, with the descriptor's code-entry offset (bytes 16..23,
which depend only on where the kernel sits in its code object) cleared.
Comments, renames and changes to other kernels leave it alone; any change to
the kernel's instructions or resources changes it.  A counter record names
the id it was taken on, and a reading is used only while that id is the one
built (bench.py reports null otherwise).

The ids are read from libzmc.so itself: its .hip_fatbin section holds one
offload bundle per translation unit ("__CLANG_OFFLOAD_BUNDLE__", entry count,
then offset, size and target triple per entry), whose gfx950 entries are the
ELF code objects.
"""
import hashlib
import os
import struct

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libzmc.so")
TARGET = "amdgcn-amd-amdhsa--gfx950"
_MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"


def _sections(data):
    """{name: (addr, offset, size, type, link)} of a little-endian ELF64 image."""
    if data[:4] != b"\x7fELF" or data[4] != 2 or data[5] != 1:
        raise ValueError("not a little-endian ELF64 image")
    shoff, = struct.unpack_from("<Q", data, 0x28)
    shentsize, shnum, shstrndx = struct.unpack_from("<HHH", data, 0x3A)
    raw = [struct.unpack_from("<IIQQQQIIQQ", data, shoff + i * shentsize) for i in range(shnum)]
    names = raw[shstrndx][4]

    def name(off):
        end = data.index(b"\0", names + off)
        return data[names + off:end].decode()

    return [(name(r[0]), r[3], r[4], r[5], r[1], r[6]) for r in raw]


def _code_object_kernels(co):
    """{mangled kernel name: id} of one gfx950 code object."""
    secs = _sections(co)
    symtab = next(s for s in secs if s[4] == 2)  # SHT_SYMTAB
    strtab = secs[symtab[5]]
    syms = {}
    for off in range(symtab[2], symtab[2] + symtab[3], 24):
        st_name, st_info, _, st_shndx, st_value, st_size = struct.unpack_from("<IBBHQQ", co, off)
        end = co.index(b"\0", strtab[2] + st_name)
        syms[co[strtab[2] + st_name:end].decode()] = (st_info & 0xF, st_shndx, st_value, st_size)

    def body(sym):
        _, shndx, value, size = sym
        _, addr, offset, _, _, _ = secs[shndx]
        start = offset + (value - addr)
        return co[start:start + size]

    out = {}
    for name, sym in syms.items():
        kd = syms.get(name + ".kd")
        if sym[0] != 2 or kd is None:  # kernels: STT_FUNC with a descriptor
            continue
        desc = bytearray(body(kd))
        desc[16:24] = b"\0" * 8
        out[name] = hashlib.sha256(body(sym) + bytes(desc)).hexdigest()[:16]
    return out


def kernel_ids(lib=LIB):
    """{mangled kernel name: id} for every kernel built into `lib`."""
    with open(lib, "rb") as fh:
        data = fh.read()
    fatbin = next((s for s in _sections(data) if s[0] == ".hip_fatbin"), None)
    if fatbin is None:
        raise ValueError(f"{lib} has no .hip_fatbin section")
    blob = data[fatbin[2]:fatbin[2] + fatbin[3]]
    out = {}
    pos = blob.find(_MAGIC)
    while pos >= 0:
        count, = struct.unpack_from("<Q", blob, pos + len(_MAGIC))
        p = pos + len(_MAGIC) + 8
        for _ in range(count):
            off, size, tlen = struct.unpack_from("<QQQ", blob, p)
            triple = blob[p + 24:p + 24 + tlen].decode()
            p += 24 + tlen
            if triple.endswith(TARGET) and size > 0:
                out.update(_code_object_kernels(blob[pos + off:pos + off + size]))
        pos = blob.find(_MAGIC, pos + 1)
    return out


def kernel_id(mangled, lib=LIB):
    """The id of one kernel (None when the library has no such kernel)."""
    return kernel_ids(lib).get(mangled)


# Mangled names of the kernels that the benchmark reports on.
GAUSS_F32_N3_POINT_MAJOR = "_ZN3zmc13k_point_majorINS_5GaussIfLi3EEEfLi3EEEvNS_10ScanParamsE"
GAUSS_F64_N3_POINT_MAJOR = "_ZN3zmc13k_point_majorINS_5GaussIdLi3EEEdLi3EEEvNS_10ScanParamsE"
COSEXP_F32_N2_POINT_MAJOR = "_ZN3zmc13k_point_majorINS_6CosExpIfLi2EEEfLi2EEEvNS_10ScanParamsE"
COSEXP_F64_N2_POINT_MAJOR = "_ZN3zmc13k_point_majorINS_6CosExpIdLi2EEEdLi2EEEvNS_10ScanParamsE"
