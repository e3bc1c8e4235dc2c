"""The pipelined element loads of the paired-store DG kernels are issued as
inline-asm vector loads that the compiler does not track: it must not read,
copy or overwrite their destination registers before the explicit wait.
Compile the forward kernels for gfx950 (no GPU needed) and scan each paired
instance's assembly: between a global load and the next `s_waitcnt vmcnt`,
no other instruction may touch the registers that load writes."""
import glob
import os
import re
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1904_09538_amd", "csrc", "dg_forward.hip")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _regs(tok):
    out = set()
    for m in re.finditer(r"\bv\[(\d+):(\d+)\]|\bv(\d+)\b", tok):
        if m.group(3):
            out.add(int(m.group(3)))
        else:
            out.update(range(int(m.group(1)), int(m.group(2)) + 1))
    return out


def _violations(body):
    """Instructions that use a register with a global load still in flight
    (straight-line scan; every wait on the vector memory counter ends the
    in-flight set, as the kernels' waits are placed to complete the loads)."""
    pending, bad = set(), []
    for line in body:
        t = line.split(";")[0].strip()
        if not t or t.startswith(".") or t.endswith(":"):
            continue
        op = t.split()[0]
        args = t[len(op):].split(",")
        if op == "s_waitcnt" and "vmcnt" in t:
            pending.clear()
            continue
        if op.startswith("global_load"):
            if set().union(*[_regs(a) for a in args[1:]]) & pending:
                bad.append(t)
            pending |= _regs(args[0])
            continue
        if args and set().union(*[_regs(a) for a in args]) & pending:
            bad.append(t)
    return bad


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_pipelined_loads_registers_untouched_until_wait():
    tmp = tempfile.mkdtemp(prefix="dgisa_")
    try:
        cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
               "-Xclang", "-packed-fp32-ops", "-c", SRC, "--save-temps", "-o", os.path.join(tmp, "f.o")]
        r = subprocess.run(cmd, cwd=tmp, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        asm = open(glob.glob(os.path.join(tmp, "*gfx950.s"))[0]).read()
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    names = [m.group(1) for m in re.finditer(r"^(_Z\S*dg_kernelIf\S*ELb0ELb1E\S*):", asm, re.M)]
    assert len(names) >= 40  # every paired FP32 instance (KQ x column blocks)
    checked = 0
    for name in names:
        i = asm.index(name + ":")
        body = asm[i:asm.index(".Lfunc_end", i)].splitlines()
        bad = _violations(body)
        assert not bad, (name, bad[:5])
        checked += 1
    assert checked == len(names)


def test_scanner_flags_early_use():
    """The scan itself: a copy of a register whose load is in flight is
    flagged; the same copy after the wait, or a use of other registers, is
    not."""
    early = ["global_load_dwordx4 v[0:3], v[8:9], off", "v_accvgpr_write_b32 a25, v2",
             "s_waitcnt vmcnt(0)"]
    late = ["global_load_dwordx4 v[0:3], v[8:9], off", "v_mov_b32_e32 v4, v5", "s_waitcnt vmcnt(4)",
            "v_mov_b32_e32 v6, v2"]
    overwrite = ["global_load_dwordx4 v[0:3], v[8:9], off", "v_mov_b32_e32 v1, 0"]
    assert _violations(early) == ["v_accvgpr_write_b32 a25, v2"]
    assert _violations(late) == []
    assert _violations(overwrite) == ["v_mov_b32_e32 v1, 0"]
