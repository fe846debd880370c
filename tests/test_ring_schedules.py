"""Host-side replay of the LDS rings' index and timing arithmetic in the
wave-per-pair kernels, with the constants read from the kernel sources:

- the wave-per-pair kernels' per-wave ring (residue codes, lane-0 feeds and
  the last-lane outputs share 638 words through overlapping arrays; the int32
  kernel leaves the second residue array unused);
- the pipelined traceback kernel's pass-boundary ring (one wave per pass,
  a fixed lag between passes, a barrier after every 64-step block).

Each check is a property the kernels rely on for correctness and that no GPU
test can isolate: every access stays inside the wave's ring, a read sees the
value of the row it needs, and no slot is overwritten before it is read."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1404_4152_amd", "csrc")


def _consts(path, names):
    text = open(os.path.join(CSRC, path)).read()
    out = {}
    for n in names:
        m = re.search(r"\b" + n + r"\s*=\s*(\d+)", text)
        assert m, f"{n} not found in {path}"
        out[n] = int(m.group(1))
    return out


RING = _consts("sw_kernels.hip", ["kRingA", "kRingB", "kRingH", "kRingF", "kRingOH", "kRingOF"])
PIPE = _consts("sw_internal.h", ["kAlignPipeRing", "kAlignPipeLag", "kAlignPipeMax"])


def _ring_words():
    text = open(os.path.join(CSRC, "sw_kernels.hip")).read()
    m = re.search(r"kRing2Bytes\s*=\s*(\d+)\s*\*\s*4", text)
    assert m
    return int(m.group(1))


def test_ring_reads_stay_in_bounds_and_hit_kept_entries():
    """At step 64b + u lane l reads entry e = 64 + u - l of every array (all
    lanes, 0 <= u, l < 64).  The word stays inside the ring; lane 0's H and F
    entries and every lane's residue entries are ones the array keeps (A, B:
    0..127; H, F: 64..127); an entry an array does not keep is only read by a
    lane > 0 for H or F, whose value the wave shift discards."""
    words = _ring_words()
    keep = {"kRingA": range(0, 128), "kRingB": range(0, 128),
            "kRingH": range(64, 128), "kRingF": range(64, 128)}
    for u in range(64):
        for l in range(64):
            e = 64 + u - l
            assert 1 <= e <= 127
            for name, kept in keep.items():
                w = RING[name] + e
                assert 0 <= w < words, (name, u, l)
                if e not in kept:
                    assert name in ("kRingH", "kRingF") and l > 0


def test_ring_arrays_do_not_overlap_where_kept_or_written():
    """Kept entries of the input arrays and written entries of the output
    arrays (1..127, every lane writes) never share a word."""
    words = _ring_words()
    owned = {}
    spans = {"kRingA": range(0, 128), "kRingB": range(0, 128), "kRingH": range(64, 128),
             "kRingF": range(64, 128), "kRingOH": range(1, 128), "kRingOF": range(1, 128)}
    for name, entries in spans.items():
        for e in entries:
            w = RING[name] + e
            assert 0 <= w < words
            assert w not in owned, (name, e, owned.get(w))
            owned[w] = name


def test_ring_output_entry_is_lane_63s_at_block_end():
    """Every lane writes its outputs of step t to entry 64 + (t mod 64) - l.
    At the end of a 64-step block, entries 1..64 must hold lane 63's values of
    that block, in row order (entry p: the row lane 63 produced at step p - 1
    of the block)."""
    last = {}
    for u in range(64):
        for l in range(64):
            last[64 + u - l] = (u, l)          # later writes of the block win
    for p in range(1, 65):
        u, l = last[p]
        assert l == 63 and u == p - 1, (p, u, l)


@pytest.mark.parametrize("P", [2, 3, 9, 12, 16])
@pytest.mark.parametrize("n", [1, 63, 64, 65, 200, 257, 1000])
def test_pipelined_traceback_ring_order(P, n):
    """Wave w runs pass w kAlignPipeLag steps behind wave w - 1, in blocks of
    64 steps separated by a workgroup barrier.  Lane 63 of wave w - 1 writes
    row r (r < n) at its step r + 63; wave w reads rows 64b..64b+63 at the
    start of its block b.  Each row is written in an earlier global block than
    the one that reads it, and the slot's next write (row r + ring) comes in a
    later global block than that read."""
    ring, lag = PIPE["kAlignPipeRing"], PIPE["kAlignPipeLag"]
    assert P <= PIPE["kAlignPipeMax"] and lag % 64 == 0 and ring % 64 == 0
    lagb = lag // 64
    steps = n + 63
    nlb = (steps + 63) // 64
    for w in range(1, P):
        # global step of wave v's local step t: t + v * lag
        for r in range(n):
            t_write = r + 63
            assert t_write < steps                       # the producer reaches it
            g_write_block = (t_write + (w - 1) * lag) // 64
            b = r // 64
            assert b < nlb
            g_read_block = b + w * lagb
            assert g_write_block < g_read_block, (w, r)
            r_next = r + ring
            if r_next < n:
                g_next_block = (r_next + 63 + (w - 1) * lag) // 64
                assert g_next_block > g_read_block, (w, r)


def test_pipelined_traceback_lds_budget():
    """The plan's LDS formula (int8 profiles, P - 1 rings, the reduction) at
    the protein alphabet: T = 4 up to 16 passes and T = 8 up to 12 fit one
    workgroup's LDS."""
    ring = PIPE["kAlignPipeRing"]

    def lds(R, T, P):
        return P * R * (64 * T + 16) + (P - 1) * ring * 8 + 3 * P * 4

    cap = 160 * 1024 - 64
    assert lds(21, 4, 16) <= cap and lds(21, 8, 12) <= cap < lds(21, 8, 13)
