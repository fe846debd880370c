"""CPU model of the narrow lane tiers' exactness argument (no GPU).

The lane-per-subject and packed wave-per-pair kernels evaluate every cell as
    h = max(hdiag + s, e, f); t = h - beta; e' = max(e - alpha, t, 0);
    f' = max(f - alpha, t, 0); best = max(best, h)
in packed fp16 (exact for integers in [-2048, 2048], threshold 1920, alpha and
beta clamped to 2048) or in saturating int16 (threshold 32767, clamp 32767).
The claim: a lane whose best stays below the threshold holds the exact score,
and a lane whose exact score reaches the threshold is flagged (its computed
best reaches the threshold too).  This model replays that arithmetic, cell
order and all, in numpy float16 / int16, vectorised over many pairs of equal
shape, and checks the claim against the oracle, including scores far beyond
the fp16 and int16 ranges and penalties beyond the clamps.  It shares no code
with the kernels or the oracle; it is a model of the design, written from the
same recurrence (section II.A, Eq. 1).
"""
import numpy as np
import pytest

import oracle


def model_f16(Q, S, M, alpha, beta):
    """Q: (B, m) codes, S: (B, n) codes; returns the fp16 best per pair."""
    B, m = Q.shape
    n = S.shape[1]
    f16 = np.float16
    na, nb = f16(-min(alpha, 2048)), f16(-min(beta, 2048))
    zero = np.zeros(B, f16)
    H = np.zeros((m, B), f16)
    E = np.zeros((m, B), f16)
    best = np.zeros(B, f16)
    Mf = M.astype(f16)
    with np.errstate(over="ignore", invalid="ignore"):
        for i in range(n):
            hdiag = zero.copy()
            f = zero.copy()
            s_col = S[:, i]
            for j in range(m):
                sc = Mf[Q[:, j], s_col]
                hold = H[j].copy()
                h = np.maximum(np.maximum(hdiag + sc, E[j]), f)
                t = h + nb
                E[j] = np.maximum(np.maximum(E[j] + na, t), zero)
                f = np.maximum(np.maximum(f + na, t), zero)
                H[j] = h
                hdiag = hold
                best = np.maximum(best, h)
    assert not np.isnan(best).any()
    return best


def model_i16(Q, S, M, alpha, beta):
    """Saturating int16 with unsigned saturating subtraction for the gap terms."""
    B, m = Q.shape
    n = S.shape[1]
    a, b = min(alpha, 32767), min(beta, 32767)
    sat = lambda x: np.clip(x, -32768, 32767)
    H = np.zeros((m, B), np.int64)
    E = np.zeros((m, B), np.int64)
    best = np.zeros(B, np.int64)
    for i in range(n):
        hdiag = np.zeros(B, np.int64)
        f = np.zeros(B, np.int64)
        s_col = S[:, i]
        for j in range(m):
            sc = M[Q[:, j], s_col].astype(np.int64)
            hold = H[j].copy()
            h = np.maximum(np.maximum(sat(hdiag + sc), E[j]), f)
            t = np.maximum(h - b, 0)
            E[j] = np.maximum(np.maximum(E[j] - a, 0), t)
            f = np.maximum(np.maximum(f - a, 0), t)
            H[j] = h
            hdiag = hold
            best = np.maximum(best, h)
    return best


def check_claim(orc, Q, S, M, alpha, beta, thr, tier):
    best = model_f16(Q, S, M, alpha, beta) if tier == "f16" else model_i16(Q, S, M, alpha, beta)
    for x in range(Q.shape[0]):
        exact = orc.sw_score(Q[x], S[x], M, alpha, beta)
        flagged = not (float(best[x]) < thr)
        assert flagged == (exact >= thr), (tier, thr, exact, float(best[x]))
        if not flagged:
            assert int(best[x]) == exact, (tier, thr, exact, float(best[x]))


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


@pytest.mark.parametrize("thr", [1920, 700, 150, 40, 9])
def test_f16_tier_random(orc, thr):
    rng = np.random.Generator(np.random.PCG64(thr))
    for A, lo, hi, L in [(20, -4, 11, 40), (6, -20, 40, 30), (4, -127, 127, 25)]:
        M = rng.integers(lo, hi + 1, size=(A, A)).astype(np.int8)
        Q = rng.integers(0, A, size=(64, L)).astype(np.uint8)
        S = rng.integers(0, A, size=(64, L + 7)).astype(np.uint8)
        for alpha, beta in [(2, 12), (0, 0), (1, 3000), (2500, 9000)]:
            check_claim(orc, Q, S, M, alpha, beta, thr, "f16")


def test_f16_tier_scores_beyond_range(orc):
    """Identical or near-identical sequences under a high diagonal: scores run
    from below 1920 to far beyond 2048 (and beyond the fp16 maximum, where the
    model reaches +inf); every such lane must be flagged."""
    rng = np.random.Generator(np.random.PCG64(3))
    A = 5
    M = np.full((A, A), -3, np.int8)
    np.fill_diagonal(M, 127)
    base = rng.integers(0, A, size=(48, 40)).astype(np.uint8)
    Q = base.copy()
    S = base.copy()
    S[::3, ::5] = (S[::3, ::5] + 1) % A      # some mismatches, some pairs exact copies
    Q[1::4, :25] = rng.integers(0, A, size=(12, 25))
    check_claim(orc, Q, S, M, 2, 12, 1920, "f16")
    # many rows: H climbs past 65504 in fp16 (inf), still flagged, never NaN
    Qb = np.tile(np.arange(A, dtype=np.uint8), (4, 120))[:, :600]
    check_claim(orc, Qb, Qb.copy(), M, 2, 12, 1920, "f16")


@pytest.mark.parametrize("thr", [32767, 5000, 60])
def test_i16_tier(orc, thr):
    rng = np.random.Generator(np.random.PCG64(thr + 1))
    A = 5
    M = rng.integers(-30, 127, size=(A, A)).astype(np.int8)
    np.fill_diagonal(M, 127)
    Q = rng.integers(0, A, size=(32, 30)).astype(np.uint8)
    S = Q.copy()
    S[::2] = rng.integers(0, A, size=(16, 30))
    for alpha, beta in [(2, 12), (0, 40000), (33000, 33000)]:
        check_claim(orc, Q, S, M, alpha, beta, thr, "i16")
    # exact copies of 300 residues at 127 each: 38,100 > 32,767
    Qb = rng.integers(0, A, size=(4, 300)).astype(np.uint8)
    Mb = np.full((A, A), -5, np.int8)
    np.fill_diagonal(Mb, 127)
    check_claim(orc, Qb, Qb.copy(), Mb, 2, 12, 32767, "i16")


def test_model_rejects_an_invalid_fp16_threshold(orc):
    """Negative control: with a threshold above the fp16 exact range the claim
    must fail on scores past 2048, so the check above has teeth."""
    A = 5
    M = np.full((A, A), -3, np.int8)
    np.fill_diagonal(M, 127)
    rng = np.random.Generator(np.random.PCG64(3))
    base = rng.integers(0, A, size=(48, 40)).astype(np.uint8)
    Q = base.copy()
    S = base.copy()
    S[::3, ::5] = (S[::3, ::5] + 1) % A
    Q[1::4, :25] = rng.integers(0, A, size=(12, 25))   # scores between 2048 and 4000 round in fp16
    with pytest.raises(AssertionError):
        check_claim(orc, Q, S, M, 2, 12, 4000, "f16")
