"""The built kernels keep clear of the wide-store data hazard of gfx950.

A buffer store of more than 64 bits reads its data registers after it has
issued; when the instruction right after it rewrites one of them, some
lanes store the new value (seen on the hardware: lanes 12..15 of every 16
stored the address the next instruction computed into the first data
register).  The compiler separates the two by a wait state only when the
store's SGPR offset field is unused, so the kernels put the whole offset of
such a store in its VGPR operand.  This test disassembles the gfx950 code
objects of the built library and checks both rules: no wide buffer store
with an SGPR offset, and no wide store (buffer or global) whose data
registers the next instruction writes."""
import os
import re
import subprocess

import pytest

import paper_1505_03271_amd as lb

LLVM = "/opt/rocm/llvm/bin"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"
WIDE = re.compile(r"^\s*(buffer_store_dwordx[34]|global_store_dwordx[34]|flat_store_dwordx[34])\s+(.*)$")


def _regs(op):
    m = re.match(r"v\[(\d+):(\d+)\]", op)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"v(\d+)$", op)
    return {int(m.group(1))} if m else set()


def _instructions(text):
    """(kernel, instruction) pairs of an llvm-objdump listing."""
    kernel = None
    for line in text.splitlines():
        m = re.match(r"^[0-9a-f]+ <(\S+)>:", line)
        if m:
            kernel = m.group(1)
            continue
        ins = line.split("//")[0].strip()
        if ins and kernel and not ins.endswith(":"):
            yield kernel, ins


def _code_objects(tmp_path):
    lib = lb.LIB_PATH
    if not os.path.exists(lib):
        pytest.skip("library not built")
    for tool in ("llvm-objcopy", "clang-offload-bundler", "llvm-objdump"):
        if not os.path.exists(os.path.join(LLVM, tool)):
            pytest.skip(f"{tool} not installed")
    fat = tmp_path / "fat.bin"
    subprocess.run([os.path.join(LLVM, "llvm-objcopy"), f"--dump-section=.hip_fatbin={fat}", lib,
                    str(tmp_path / "lib.copy")], check=True, capture_output=True)
    data = fat.read_bytes()
    starts = [m.start() for m in re.finditer(re.escape(MAGIC), data)] + [len(data)]
    assert len(starts) > 1, "no offload bundle in the library"
    listings = []
    for q in range(len(starts) - 1):
        part = tmp_path / f"bundle{q}.bin"
        part.write_bytes(data[starts[q]:starts[q + 1]])
        co = tmp_path / f"co{q}.elf"
        r = subprocess.run([os.path.join(LLVM, "clang-offload-bundler"), "--unbundle", "--type=o",
                            f"--input={part}", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={co}"],
                           capture_output=True, text=True)
        if r.returncode != 0 or not co.exists() or co.stat().st_size == 0:
            continue
        dis = subprocess.run([os.path.join(LLVM, "llvm-objdump"), "-d", "--mcpu=gfx950", str(co)],
                             check=True, capture_output=True, text=True).stdout
        listings.append(dis)
    assert listings, "no gfx950 code object in the library"
    return listings


def _hazards(text):
    """(number of wide stores, problems) of one listing."""
    ins = list(_instructions(text))
    wide = 0
    problems = []
    for k, (kernel, line) in enumerate(ins):
        m = WIDE.match(line)
        if not m:
            continue
        wide += 1
        ops = [o.strip() for o in m.group(2).split(",")]
        if m.group(1).startswith("buffer"):
            data, soff = _regs(ops[0]), ops[3].split()[0]
            if soff.startswith("s"):
                problems.append(f"{kernel}: SGPR offset: {line}")
        else:
            data = _regs(ops[1])
        if k + 1 < len(ins) and ins[k + 1][0] == kernel:
            nxt = ins[k + 1][1]
            w = re.match(r"(v_\S+)\s+(v\[\d+:\d+\]|v\d+)", nxt)
            if w and _regs(w.group(2)) & data:
                problems.append(f"{kernel}: data rewritten at once: {line} / {nxt}")
    return wide, problems


def test_no_wide_store_data_hazard(tmp_path):
    wide = 0
    problems = []
    for text in _code_objects(tmp_path):
        n, p = _hazards(text)
        wide += n
        problems += p
    assert wide > 0, "no wide store found: the listing was not parsed"
    assert not problems, "\n".join(problems[:20])


def test_scanner_catches_the_hazard():
    """The check itself: the pattern seen on the hardware is flagged, the
    same store with a wait state and no SGPR offset is not."""
    text = ("0000000000001000 <_Zkernel>:\n"
            "\tbuffer_store_dwordx4 v[14:17], v18, s[56:59], s9 offen // 000000001000: E07C\n"
            "\tv_add_u32_e32 v14, s87, v72 // 000000001008: 681C\n"
            "\tbuffer_store_dwordx4 v[20:23], v18, s[56:59], 0 offen // 00000000100C: E07C\n"
            "\ts_nop 0 // 000000001014: BF80\n"
            "\tv_add_u32_e32 v20, s87, v72 // 000000001018: 681C\n"
            "\tglobal_store_dwordx4 v[0:1], v[30:33], off // 00000000101C: DC7C\n"
            "\tv_mov_b32_e32 v31, 0 // 000000001024: 7E3E\n")
    wide, problems = _hazards(text)
    assert wide == 3
    assert len(problems) == 3, problems
    assert "SGPR offset" in problems[0] and "v[14:17]" in problems[0]
    assert "rewritten" in problems[1] and "v[14:17]" in problems[1]
    assert "rewritten" in problems[2] and "global_store" in problems[2]
