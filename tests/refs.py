"""Independent references that pin the CPU oracle (tests only).

None of these re-types Eq. 1.  Each computes the local-alignment score from a
different definition or algorithm, so that a dropped term, a wrong sign, a
wrong index or a transposed matrix in the oracle disagrees with at least one:

* ``brute_force``: the plain definition.  Enumerate every alignment of every
  pair of substrings (all match / gap column sequences), score each one by
  summing substitution scores and charging every maximal run of k gap columns
  in the same sequence beta + (k-1)*alpha (section II.A: beta = open +
  extension, alpha = extension), and take the maximum together with 0 (the
  empty alignment).  Exponential; |q|, |s| <= 5.
* ``general_gap_dp``: the cubic Waterman-Smith-Beyer recurrence with an
  arbitrary gap-length cost g(k) = beta + (k-1)*alpha.
* ``linear_gap_sw``: the textbook linear-gap Smith-Waterman recurrence; the
  affine model reduces to it when alpha == beta.
* ``ungapped``: the best ungapped local alignment (Kadane along every
  diagonal); the affine model reduces to it when gaps cost more than any
  alignment can gain.

Orientation throughout: the substitution score of query residue a against
subject residue b is ``M[a][b]`` (matrix row = query residue).
"""
from __future__ import annotations

import numpy as np


def _score_columns(cols, q, s, M, alpha, beta):
    """Score one alignment given as a list of columns.

    A column is ('M', qi, sj), ('Q', qi) (query residue against a gap) or
    ('S', sj) (subject residue against a gap).
    """
    total = 0
    run_kind, run_len = None, 0
    for col in cols + [("END",)]:
        kind = col[0]
        if kind in ("Q", "S") and kind == run_kind:
            run_len += 1
            continue
        if run_kind is not None:
            total -= beta + (run_len - 1) * alpha
            run_kind, run_len = None, 0
        if kind == "M":
            total += int(M[q[col[1]]][s[col[2]]])
        elif kind in ("Q", "S"):
            run_kind, run_len = kind, 1
    return total


def _alignments(qa, qb, sa, sb):
    """Every global alignment of q[qa:qb] with s[sa:sb] as a column list."""
    if qa == qb and sa == sb:
        yield []
        return
    if qa < qb and sa < sb:
        for rest in _alignments(qa + 1, qb, sa + 1, sb):
            yield [("M", qa, sa)] + rest
    if qa < qb:
        for rest in _alignments(qa + 1, qb, sa, sb):
            yield [("Q", qa)] + rest
    if sa < sb:
        for rest in _alignments(qa, qb, sa + 1, sb):
            yield [("S", sa)] + rest


def brute_force(q, s, M, alpha, beta):
    """Maximum over all local alignments (and the empty one) by enumeration."""
    q = [int(x) for x in q]
    s = [int(x) for x in s]
    best = 0
    m, n = len(q), len(s)
    for qa in range(m):
        for qb in range(qa + 1, m + 1):
            for sa in range(n):
                for sb in range(sa + 1, n + 1):
                    for cols in _alignments(qa, qb, sa, sb):
                        v = _score_columns(cols, q, s, M, alpha, beta)
                        if v > best:
                            best = v
    return best


def general_gap_table(q, s, M, alpha, beta):
    """Cubic local-alignment DP with gap cost g(k) = beta + (k-1)*alpha.
    Returns V with V[a][b] = best score of a local alignment ending at query
    residue a and subject residue b (1-based; 0 = none)."""
    m, n = len(q), len(s)

    def g(k):
        return beta + (k - 1) * alpha

    V = [[0] * (n + 1) for _ in range(m + 1)]
    for a in range(1, m + 1):
        for b in range(1, n + 1):
            v = max(0, V[a - 1][b - 1] + int(M[int(q[a - 1])][int(s[b - 1])]))
            for k in range(1, a + 1):          # run of k query residues against gaps
                v = max(v, V[a - k][b] - g(k))
            for k in range(1, b + 1):          # run of k subject residues against gaps
                v = max(v, V[a][b - k] - g(k))
            V[a][b] = v
    return V


def general_gap_dp(q, s, M, alpha, beta):
    """Best score of the cubic recurrence (max over general_gap_table)."""
    V = general_gap_table(q, s, M, alpha, beta)
    return max([0] + [v for row in V for v in row])


def alignment_columns(al):
    """Columns of an alignment given as begin positions and (op, length) runs:
    op 0 aligned pair, 1 query residue against a gap, 2 subject residue
    against a gap."""
    qi, sj = al["q_begin"], al["s_begin"]
    cols = []
    for op, k in al["ops"]:
        for _ in range(k):
            if op == 0:
                cols.append(("M", qi, sj))
                qi += 1
                sj += 1
            elif op == 1:
                cols.append(("Q", qi))
                qi += 1
            else:
                cols.append(("S", sj))
                sj += 1
    return cols, qi, sj


def score_alignment(al, q, s, M, alpha, beta):
    """Score of an alignment by the run-cost definition (as brute_force)."""
    cols, _, _ = alignment_columns(al)
    return _score_columns(cols, q, s, M, alpha, beta)


def linear_gap_sw(q, s, M, d):
    """Textbook Smith-Waterman with a linear gap penalty d per gap column."""
    m, n = len(q), len(s)
    V = np.zeros((m + 1, n + 1), dtype=np.int64)
    for a in range(1, m + 1):
        for b in range(1, n + 1):
            V[a, b] = max(0, V[a - 1, b - 1] + int(M[int(q[a - 1])][int(s[b - 1])]),
                          V[a - 1, b] - d, V[a, b - 1] - d)
    return int(V.max()) if V.size else 0


def ungapped(q, s, M):
    """Best ungapped local alignment: Kadane's maximum subarray on each diagonal."""
    m, n = len(q), len(s)
    best = 0
    for off in range(-(m - 1), n):
        run = 0
        for a in range(m):
            b = a + off
            if 0 <= b < n:
                run = max(0, run + int(M[int(q[a])][int(s[b])]))
                best = max(best, run)
    return best
