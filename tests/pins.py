"""Pins for the CPU oracle: each check compares the oracle with something the
paper or the mathematics fixes, never with a re-typed copy of Eq. 1.

Every check takes an ``oracle.Oracle`` and returns a list of failure strings
(empty = pass).  ``tests/test_oracle_pins.py`` runs them on the real oracle;
``tests/test_oracle_mutants.py`` runs them on oracles with planted mistakes
and requires every mistake to be caught by at least one check.
"""
from __future__ import annotations

import functools
import os

import numpy as np

import refs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.txt")
_LETTERS = {"A": 0, "C": 1, "G": 2}


def load_golden():
    cases = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, q, s, match, mismatch, alpha, beta, exp = line.split()
            enc = (lambda x: np.array([], np.uint8) if x == "-"
                   else np.array([_LETTERS[c] for c in x], np.uint8))
            M = np.full((3, 3), int(mismatch), np.int8)
            np.fill_diagonal(M, int(match))
            cases.append((name, enc(q), enc(s), M, int(alpha), int(beta), int(exp)))
    return cases


def tiny_cases(n=260, max_len=5, seed=11):
    """Random tiny cases (alphabet 2-4, asymmetric matrices, 0 <= alpha <= beta)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for t in range(n):
        A = int(rng.integers(2, 5))
        M = rng.integers(-5, 6, size=(A, A)).astype(np.int8)
        lq = int(rng.integers(0 if t % 17 == 0 else 1, max_len + 1))
        ls = int(rng.integers(0 if t % 13 == 0 else 1, max_len + 1))
        if lq * ls > 20:            # keep the enumeration affordable
            ls = max(1, 20 // max(lq, 1))
        q = rng.integers(0, A, size=lq).astype(np.uint8)
        s = rng.integers(0, A, size=ls).astype(np.uint8)
        beta = int(rng.integers(0, 8))
        alpha = int(rng.integers(0, beta + 1))
        out.append((q, s, M, alpha, beta))
    return out


def mid_cases(n=60, max_len=14, seed=12):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n):
        A = int(rng.integers(2, 6))
        M = rng.integers(-6, 7, size=(A, A)).astype(np.int8)
        q = rng.integers(0, A, size=int(rng.integers(1, max_len + 1))).astype(np.uint8)
        s = rng.integers(0, A, size=int(rng.integers(1, max_len + 1))).astype(np.uint8)
        beta = int(rng.integers(0, 12))
        alpha = int(rng.integers(0, beta + 1))
        out.append((q, s, M, alpha, beta))
    return out


@functools.lru_cache(maxsize=None)
def _brute_table():
    return [refs.brute_force(q, s, M, a, b) for (q, s, M, a, b) in tiny_cases()]


@functools.lru_cache(maxsize=None)
def _cubic_table():
    return [refs.general_gap_dp(q, s, M, a, b) for (q, s, M, a, b) in mid_cases()]


def check_golden(o):
    fails = []
    for name, q, s, M, a, b, exp in load_golden():
        got = o.sw_score(q, s, M, a, b)
        if got != exp:
            fails.append(f"golden {name}: got {got}, expected {exp}")
    return fails


def check_orientation(o):
    """Matrix row = query residue (the query profile's orientation)."""
    fails = []
    M = np.array([[0, 5], [-3, 0]], np.int8)
    got = o.sw_score(np.array([0], np.uint8), np.array([1], np.uint8), M, 1, 3)
    if got != 5:
        fails.append(f"orientation: q=(0) s=(1) M=[[0,5],[-3,0]] gave {got}, expected 5")
    got = o.sw_score(np.array([1], np.uint8), np.array([0], np.uint8), M, 1, 3)
    if got != 0:
        fails.append(f"orientation: q=(1) s=(0) gave {got}, expected 0")
    return fails


def check_brute_force(o):
    fails = []
    for (q, s, M, a, b), exp in zip(tiny_cases(), _brute_table()):
        got = o.sw_score(q, s, M, a, b)
        if got != exp:
            fails.append(f"brute force: q={q.tolist()} s={s.tolist()} a={a} b={b} "
                         f"got {got} expected {exp}")
            if len(fails) > 5:
                break
    return fails


def check_general_gap(o):
    fails = []
    for (q, s, M, a, b), exp in zip(mid_cases(), _cubic_table()):
        got = o.sw_score(q, s, M, a, b)
        if got != exp:
            fails.append(f"cubic DP: len {len(q)}x{len(s)} a={a} b={b} got {got} expected {exp}")
            if len(fails) > 5:
                break
    return fails


def check_linear_gap(o, n=40, seed=13):
    """alpha == beta: the affine model is the linear-gap model."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fails = []
    for _ in range(n):
        A = int(rng.integers(2, 8))
        M = rng.integers(-6, 8, size=(A, A)).astype(np.int8)
        q = rng.integers(0, A, size=int(rng.integers(1, 30))).astype(np.uint8)
        s = rng.integers(0, A, size=int(rng.integers(1, 30))).astype(np.uint8)
        d = int(rng.integers(0, 9))
        exp = refs.linear_gap_sw(q, s, M, d)
        got = o.sw_score(q, s, M, d, d)
        if got != exp:
            fails.append(f"linear gap d={d}: got {got} expected {exp}")
    return fails


def check_ungapped(o, n=40, seed=14):
    """Gaps dearer than any gain: the best ungapped local alignment."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fails = []
    for _ in range(n):
        A = int(rng.integers(2, 8))
        M = rng.integers(-6, 8, size=(A, A)).astype(np.int8)
        q = rng.integers(0, A, size=int(rng.integers(1, 30))).astype(np.uint8)
        s = rng.integers(0, A, size=int(rng.integers(1, 30))).astype(np.uint8)
        beta = 8 * 30 + 1
        alpha = int(rng.integers(0, beta + 1))
        exp = refs.ungapped(q, s, M)
        got = o.sw_score(q, s, M, alpha, beta)
        if got != exp:
            fails.append(f"ungapped: got {got} expected {exp}")
    return fails


def _rand_case(rng, max_len=40, A=None, sym=False):
    A = A or int(rng.integers(2, 21))
    M = rng.integers(-5, 9, size=(A, A)).astype(np.int8)
    if sym:
        M = (np.triu(M) + np.triu(M, 1).T).astype(np.int8)
    q = rng.integers(0, A, size=int(rng.integers(1, max_len))).astype(np.uint8)
    s = rng.integers(0, A, size=int(rng.integers(1, max_len))).astype(np.uint8)
    beta = int(rng.integers(0, 15))
    alpha = int(rng.integers(0, beta + 1))
    return q, s, M, alpha, beta


def check_invariants(o, n=60, seed=15):
    """Properties any correct local-alignment score has."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fails = []
    for t in range(n):
        q, s, M, a, b = _rand_case(rng)
        A = M.shape[0]
        v = o.sw_score(q, s, M, a, b)
        top = int(max(0, max(int(M[x][y]) for x in q for y in s)))
        if not (0 <= v <= max(0, int(M.max())) * min(len(q), len(s))):
            fails.append(f"bounds: {v}")
        if v < top:
            fails.append(f"lower bound single pair: {v} < {top}")
        # swap the sequences and transpose the matrix
        if o.sw_score(s, q, M.T.copy(), a, b) != v:
            fails.append("swap with transposed matrix")
        # reverse both sequences
        if o.sw_score(q[::-1].copy(), s[::-1].copy(), M, a, b) != v:
            fails.append("reversal")
        # dearer gaps never help
        if o.sw_score(q, s, M, a, b + 1) > v or (a < b and o.sw_score(q, s, M, a + 1, b) > v):
            fails.append("monotone in gap penalties")
        # longer subject never hurts; concatenation beats each part
        s2 = rng.integers(0, A, size=int(rng.integers(1, 20))).astype(np.uint8)
        v2 = o.sw_score(q, s2, M, a, b)
        vc = o.sw_score(q, np.concatenate([s, s2]), M, a, b)
        if vc < max(v, v2):
            fails.append("concatenated subject below a part")
        # end padding with a code that scores 0 against everything is neutral
        Mp = np.zeros((A + 1, A + 1), np.int8)
        Mp[:A, :A] = M
        pad = np.full(int(rng.integers(1, 9)), A, np.uint8)
        if o.sw_score(np.concatenate([q, pad]), np.concatenate([s, pad]), Mp, a, b) != v:
            fails.append("zero-score end padding changed the score")
        # self score of a sequence under a positive diagonal
        if (np.diag(M) > 0).all():
            sv = o.sw_score(q, q, M, a, b)
            if sv < int(sum(int(M[x][x]) for x in q)):
                fails.append("self score below its diagonal sum")
        if fails:
            break
    return fails


def check_search_driver(o, seed=16):
    """The database driver returns each sequence's own pairwise score."""
    rng = np.random.Generator(np.random.PCG64(seed))
    A = 20
    M = rng.integers(-4, 10, size=(A, A)).astype(np.int8)
    lens = rng.integers(0, 60, size=150)
    offs = np.zeros(151, np.int64)
    offs[1:] = np.cumsum(lens)
    res = rng.integers(0, A, size=int(offs[-1])).astype(np.uint8)
    q = rng.integers(0, A, size=37).astype(np.uint8)
    got = o.search(q, res, offs, M, 2, 12)
    exp = [o.sw_score(q, res[offs[k]:offs[k + 1]], M, 2, 12) for k in range(150)]
    sub = o.search_subset(q, res, offs, np.array([5, 0, 149, 5]), M, 2, 12)
    fails = []
    if got.tolist() != exp:
        fails.append("search() differs from per-pair scores")
    if sub.tolist() != [exp[5], exp[0], exp[149], exp[5]]:
        fails.append("search_subset() differs from per-pair scores")
    return fails


GOLDEN_ALIGN = os.path.join(os.path.dirname(__file__), "golden", "align_examples.txt")
_ABC = {"A": 0, "B": 1, "C": 2}
_OPS = {"M": 0, "I": 1, "D": 2}


def load_golden_align():
    import re
    cases = []
    with open(GOLDEN_ALIGN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            (name, q, s, match, mismatch, alpha, beta, score, qb, qe, sb, se,
             ops) = line.split()
            M = np.full((3, 3), int(mismatch), np.int8)
            np.fill_diagonal(M, int(match))
            exp = {"score": int(score), "q_begin": int(qb), "q_end": int(qe),
                   "s_begin": int(sb), "s_end": int(se),
                   "ops": [(_OPS[op], int(k)) for k, op in re.findall(r"(\d+)([MID])", ops)]}
            cases.append((name, np.array([_ABC[c] for c in q], np.uint8),
                          np.array([_ABC[c] for c in s], np.uint8), M, int(alpha), int(beta),
                          exp))
    return cases


def check_align_golden(o):
    """Hand-derived alignments, including every tie the traceback rules decide."""
    fails = []
    for name, q, s, M, a, b, exp in load_golden_align():
        got = o.sw_align(q, s, M, a, b)
        if got != exp:
            fails.append(f"align golden {name}: got {got}, expected {exp}")
    return fails


def _align_cases(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    cases = list(tiny_cases(n=120, seed=seed))
    for _ in range(60):
        A = int(rng.integers(2, 5))
        M = rng.integers(-6, 8, size=(A, A)).astype(np.int8)
        np.fill_diagonal(M, rng.integers(3, 9, size=A))
        q = rng.integers(0, A, size=int(rng.integers(1, 13))).astype(np.uint8)
        s = rng.integers(0, A, size=int(rng.integers(1, 13))).astype(np.uint8)
        a = int(rng.integers(0, 4))
        b = a + int(rng.integers(0, 6))
        cases.append((q, s, M, a, b))
    return cases


def check_align_rescore(o):
    """The alignment is an optimal local alignment: by the run-cost
    definition it scores the Smith-Waterman score (itself pinned above), it
    consumes exactly q[q_begin..q_end] and s[s_begin..s_end], and it begins and
    ends with an aligned pair; the empty alignment exactly when the score is 0."""
    fails = []
    for q, s, M, a, b in _align_cases(21):
        al = o.sw_align(q, s, M, a, b)
        sc = o.sw_score(q, s, M, a, b)
        if al["score"] != sc:
            fails.append(f"align score {al['score']} != sw_score {sc}")
            continue
        if sc == 0:
            if al["ops"] or al["q_begin"] != -1 or al["s_end"] != -1:
                fails.append("score 0 but a non-empty alignment")
            continue
        cols, qi, sj = refs.alignment_columns(al)
        if not (0 <= al["q_begin"] <= al["q_end"] < len(q) and 0 <= al["s_begin"] <= al["s_end"] < len(s)):
            fails.append("alignment bounds outside the sequences")
            continue
        if (qi - 1, sj - 1) != (al["q_end"], al["s_end"]):
            fails.append("alignment does not end at q_end, s_end")
            continue
        if refs.score_alignment(al, q, s, M, a, b) != sc:
            fails.append(f"alignment rescored {refs.score_alignment(al, q, s, M, a, b)} != {sc}")
        if not al["ops"] or al["ops"][0][0] != 0 or al["ops"][-1][0] != 0:
            fails.append("alignment does not begin and end with an aligned pair")
    return fails


def check_align_end(o):
    """The end cell is the first maximum of the cubic recurrence's table in
    subject-then-query order (the end-cell reading)."""
    fails = []
    for q, s, M, a, b in _align_cases(22)[::2]:
        V = refs.general_gap_table(q, s, M, a, b)
        best = max([0] + [v for row in V for v in row])
        al = o.sw_align(q, s, M, a, b)
        if best == 0:
            continue
        first = min((sb, qa) for qa in range(1, len(q) + 1) for sb in range(1, len(s) + 1)
                    if V[qa][sb] == best)
        if (al["s_end"] + 1, al["q_end"] + 1) != first:
            fails.append(f"end {(al['s_end'], al['q_end'])} != first maximum {first}")
    return fails


ALL_CHECKS = {
    "golden": check_golden,
    "orientation": check_orientation,
    "brute_force": check_brute_force,
    "general_gap": check_general_gap,
    "linear_gap": check_linear_gap,
    "ungapped": check_ungapped,
    "invariants": check_invariants,
    "search_driver": check_search_driver,
    "align_golden": check_align_golden,
    "align_rescore": check_align_rescore,
    "align_end": check_align_end,
}


def failing_checks(o):
    """Names of the checks that fail on oracle ``o``."""
    return [name for name, fn in ALL_CHECKS.items() if fn(o)]
