"""Code generation of the fp16 kernels' hot loops (CPU: hipcc cross-compiles).

gfx950 needs one wait state between a packed fp16 instruction and a packed
fp16 instruction right after it that reads its result; the compiler emits it
as ``s_nop``.  The fp16 kernels write their cell steps so that independent work
sits between the dependent ones.  This test compiles the kernel source with
the library's own flags and checks, in the largest basic block of each hot
kernel (its step loop), that the wait states stay well below what the
cell-by-cell order gave (216 per 784 VALU instructions in the lane kernel,
75 per 475 in the packed wave-per-pair kernel), and that every adjacent pair
of dependent packed instructions still carries its wait state (the rule this
relies on).
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_1404_4152_amd import build as libbuild

HIPCC = libbuild.HIPCC
KERNELS = os.path.join(libbuild.CSRC, "sw_kernels.hip")

LANE = "_ZN4swmi12inter_kernelILi32ELi4ELi1ELi16EEEvNS_9InterArgsENS_9IntraArgsEi"
PACKED = "_ZN4swmi13intra2_kernelILi16ELi4EEEvNS_9IntraArgsE"


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which(HIPCC)):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("codegen") / "k.s")
    flags = [f for f in libbuild.FLAGS if f not in ("-shared", "-fPIC", "-lpthread")]
    subprocess.run([HIPCC, *flags, "-S", "--cuda-device-only", KERNELS, "-o", out], check=True,
                   capture_output=True)
    return open(out).read().split("\n")


def blocks(lines, name):
    """Basic blocks of one function: lists of instruction lines."""
    start = next(i for i, l in enumerate(lines) if l.startswith(name + ":"))
    res, cur = [], []
    for l in lines[start + 1:]:
        if l.startswith(".Lfunc_end"):
            break
        if re.match(r"^\.LBB\S+:", l):
            res.append(cur)
            cur = []
            continue
        s = l.split(";")[0].strip()
        if s and not s.startswith("."):
            cur.append(s)
    res.append(cur)
    return res


def loop_stats(lines, name):
    body = max(blocks(lines, name), key=len)
    ops = [s.split()[0] for s in body]
    return sum(o == "s_nop" for o in ops), sum(o.startswith("v_") for o in ops)


@pytest.mark.parametrize("name,old_ratio", [(LANE, 216 / 784), (PACKED, 75 / 475)])
def test_step_loop_wait_states(asm, name, old_ratio):
    nops, valu = loop_stats(asm, name)
    assert valu > 400, (name, valu)
    assert nops / valu < 0.5 * old_ratio, (name, nops, valu)


def regs(op):
    m = re.match(r"v\[(\d+):(\d+)\]", op)
    if m:
        return {f"v{r}" for r in range(int(m.group(1)), int(m.group(2)) + 1)}
    return {op} if re.match(r"v\d+$", op) else set()


def test_dependent_packed_pairs_carry_a_wait_state(asm):
    body = max(blocks(asm, LANE), key=len)
    pairs = with_nop = 0
    prev, nop = None, False
    for s in body:
        parts = s.split(None, 1)
        op, args = parts[0], [a.strip() for a in parts[1].split(",")] if len(parts) > 1 else []
        if op == "s_nop":
            nop = True
            continue
        if prev and op.startswith("v_pk_") and args:
            dst = regs(prev[1][0])
            if dst & set().union(*[regs(a) for a in args[1:]]):
                pairs += 1
                with_nop += nop
        prev = (op, args) if op.startswith("v_pk_") else None
        nop = False
    assert pairs > 0
    assert with_nop == pairs, (with_nop, pairs)
