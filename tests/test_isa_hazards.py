"""The gfx950 code object of the built library has no store-data hazard.

A VALU instruction that writes a VGPR holding the data of an immediately
preceding vector-memory store of more than 64 bits (dwordx3 / dwordx4) needs
one wait state in between.  The compiler inserts it for the stores it emits
but not for stores written as inline asm; the library's write-through stores
are inline asm and carry their own `s_nop`.  This test disassembles the
device code object that was built here (no GPU needed) and checks every such
store against the instruction that follows it.
"""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2109_12688_amd", "libnadmm.so")
LLVM = "/opt/rocm/llvm/bin"
WIDE_STORE = re.compile(r"^(global|buffer|flat)_store_dword(x3|x4)\b")


def _vgprs(op: str):
    m = re.fullmatch(r"v\[(\d+):(\d+)\]", op)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.fullmatch(r"v(\d+)", op)
    return {int(m.group(1))} if m else set()


def _instructions(text: str):
    for line in text.splitlines():
        line = line.split("//")[0].strip()
        if not line or line.endswith(":") or line.startswith((";", ".")) or " <" in line:
            continue
        yield line


def _store_data(ins: str):
    ops = [o.strip() for o in ins.split(None, 1)[1].split(",")]
    # global/flat: vaddr, vdata, ...; buffer: vdata, vaddr, ...
    return _vgprs(ops[0] if ins.startswith("buffer_") else ops[1])


def _valu_dest(ins: str):
    if not ins.startswith("v_"):
        return set()
    parts = ins.split(None, 1)
    if len(parts) < 2:
        return set()
    return _vgprs(parts[1].split(",")[0].strip())


def hazards(disassembly: str):
    ins = list(_instructions(disassembly))
    found = []
    for a, b in zip(ins, ins[1:]):
        if WIDE_STORE.match(a) and _store_data(a) & _valu_dest(b):
            found.append((a, b))
    return found


def test_checker_finds_a_planted_hazard():
    text = ("\tglobal_store_dwordx4 v[34:35], v[30:33], off sc0 sc1\n"
            "\tv_lshl_add_u64 v[30:31], v[26:27], 2, s[22:23]\n"
            "\tglobal_store_dwordx4 v[4:5], v[0:3], off sc0 sc1\n"
            "\ts_nop 1\n"
            "\tv_mov_b32_e32 v0, 0\n"
            "\tglobal_store_dwordx2 v[4:5], v[0:1], off\n"
            "\tv_mov_b32_e32 v0, 0\n")
    assert hazards(text) == [("global_store_dwordx4 v[34:35], v[30:33], off sc0 sc1",
                              "v_lshl_add_u64 v[30:31], v[26:27], 2, s[22:23]")]


def test_library_code_objects_have_no_store_data_hazard(tmp_path):
    """Every translation unit's gfx950 code object: the .hip_fatbin section
    holds one offload bundle per source file with device code."""
    tools = [os.path.join(LLVM, t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-objdump")]
    if not os.path.exists(LIB) or not all(os.path.exists(t) for t in tools):
        pytest.skip("library not built or ROCm LLVM tools missing")
    fat = tmp_path / "fat.bin"
    subprocess.run([tools[0], f"--dump-section=.hip_fatbin={fat}", LIB], check=True)
    data = fat.read_bytes()
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    starts = [m.start() for m in re.finditer(re.escape(magic), data)]
    assert len(starts) >= 2  # kernels.hip and adjoint.hip
    n_wide = 0
    for n, (a, b) in enumerate(zip(starts, starts[1:] + [len(data)])):
        part, dev = tmp_path / f"part{n}.bin", tmp_path / f"dev{n}.o"
        part.write_bytes(data[a:b])
        subprocess.run([tools[1], "--type=o", "--unbundle", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950",
                        f"--input={part}", f"--output={dev}"], check=True)
        text = subprocess.run([tools[2], "-d", "--mcpu=gfx950", str(dev)], check=True, capture_output=True,
                              text=True).stdout
        n_wide += sum(1 for i in _instructions(text) if WIDE_STORE.match(i))
        assert hazards(text) == [], f"code object {n}"
    assert n_wide > 0
