"""Build-time check of the LDS-direct loads in the built gfx950 code.

The GEMM kernels issue ``global_load_lds_dwordx4`` from inline assembly,
which first sets M0 to the LDS destination.  The compiler treats M0 as a
reserved register, so the correctness of those kernels rests on two facts
about the code it generates, checked here on the disassembly of the library's
own objects:

1. every explicit write of M0 is the inline-assembly sequence
   ``s_mov_b32 m0, sN`` / ``s_nop 0`` / ``global_load_lds_dwordx4``;
2. no kernel that contains such a load holds any other instruction that reads
   M0 implicitly (relative register moves, messages, GWS / append / consume
   and ordered-count LDS operations, interpolation, buffer loads into LDS).

Then no compiler-made M0 value can be overwritten by the inline assembly,
and the value it writes is consumed by the very next load.
"""
from __future__ import annotations

import pathlib
import re
import subprocess
import tempfile

LLVM = pathlib.Path("/opt/rocm/llvm/bin")
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"
# instructions that read M0 without naming it
IMPLICIT_M0 = re.compile(r"^\s*(s_movrel|v_movrel|s_sendmsg|ds_gws|ds_append|ds_consume|ds_ordered_count|"
                         r"v_interp|buffer_load_\w+\s.*\blds\b|buffer_store_lds|global_load_lds_(?!dwordx4))")
FUNC = re.compile(r"^[0-9a-f]+ <(.+)>:$")


def disassemble(obj: pathlib.Path, tmp: pathlib.Path) -> str:
    fb, co = tmp / (obj.name + ".fatbin"), tmp / (obj.name + ".co")
    subprocess.run([str(LLVM / "llvm-objcopy"), f"--dump-section=.hip_fatbin={fb}", str(obj)], check=True,
                   capture_output=True)
    subprocess.run([str(LLVM / "clang-offload-bundler"), "--unbundle", "--type=o", f"--input={fb}",
                    f"--targets={TARGET}", f"--output={co}"], check=True, capture_output=True)
    r = subprocess.run([str(LLVM / "llvm-objdump"), "-d", "--no-show-raw-insn", str(co)], check=True,
                       capture_output=True, text=True)
    return r.stdout


def check_text(text: str) -> tuple[int, list[str]]:
    """(number of kernels with LDS-direct loads, problems found)."""
    funcs: dict[str, list[str]] = {}
    cur = None
    for line in text.splitlines():
        m = FUNC.match(line)
        if m:
            cur = m.group(1)
            funcs[cur] = []
        elif cur is not None and line.strip() and not line.lstrip().startswith(";"):
            funcs[cur].append(line.split("//")[0].strip())
    n, bad = 0, []
    for name, ins in funcs.items():
        if not any(i.startswith("global_load_lds_dwordx4") for i in ins):
            continue
        n += 1
        for k, i in enumerate(ins):
            if re.search(r"\bm0\b", i):
                ok = (re.match(r"^s_mov_b32 m0, s\d+$", i) and k + 2 < len(ins) and ins[k + 1] == "s_nop 0"
                      and ins[k + 2].startswith("global_load_lds_dwordx4"))
                if not ok:
                    bad.append(f"{name}: M0 used outside the load sequence: {i}")
            elif IMPLICIT_M0.match(i):
                bad.append(f"{name}: instruction that reads M0: {i}")
            elif i.startswith("global_load_lds_dwordx4") and not (k >= 2 and ins[k - 1] == "s_nop 0" and
                                                                   re.match(r"^s_mov_b32 m0, s\d+$", ins[k - 2])):
                bad.append(f"{name}: LDS-direct load without its M0 write: {i}")
    return n, bad


def check_objects(objs) -> int:
    """Raises RuntimeError on a violation; returns the number of kernels checked."""
    total, problems = 0, []
    with tempfile.TemporaryDirectory() as d:
        for obj in objs:
            obj = pathlib.Path(obj)
            if obj.suffix != ".o" or ".hip" not in obj.name:
                continue
            n, bad = check_text(disassemble(obj, pathlib.Path(d)))
            total += n
            problems += bad
    if problems:
        raise RuntimeError("LDS-direct M0 check failed:\n" + "\n".join(problems[:20]))
    return total
