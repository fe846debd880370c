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
the fp16 and int16 ranges and penalties beyond the clamps.  The lane-per-
subject fp16 tier uses a frame form of the same recurrence (cell (r, j) offset
by alpha * ((r mod 32) + (j mod 4)), so E needs no per-row decay and F one
decay per four columns); its model replays that arithmetic with strips, frame
periods and padding, against the ceiling 1920 - 36 alpha, with negative
controls at the unshifted ceiling and without the running best's last step.
It shares no code with the kernels or the oracle; it is a model of the design,
written from the same recurrence (section II.A, Eq. 1).
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


def frame_ceiling(thr, alpha, rows=32):
    """Ceiling of the packed wave-per-pair fp16 row frame for gap extension alpha."""
    if alpha > 56:
        return 0
    return min(thr, 1920 - (rows + 1) * alpha)


def lane_ceiling(thr, alpha, rows=32, G=4):
    """Ceiling of the lane-per-subject fp16 tier (row and column-class frame)
    for a query with gap extension alpha: offsets reach (rows + G - 1) alpha."""
    if (rows + G) * alpha >= 1920:
        return 0
    return min(thr, 1920 - (rows + G) * alpha)


def model_f16_frame(Q, S, M, alpha, beta, T=8, rows=32, chunk=4, G=4, extra_chunk=True,
                    tail=True):
    """Frame form of the lane-per-subject fp16 tier, replayed in numpy float16:
    the query in strips of T columns (boundary H and F of every row handed to
    the next strip), subjects padded with zero-score rows to a multiple of
    `chunk` (plus one extra chunk if `extra_chunk`), the query with zero-score
    columns to a multiple of T.  Cell (r, j) is held at offset
    alpha * ((r mod rows) + (j mod G)): E needs no per-row decay and F needs
    its decay only when j + 1 starts a new class group (by G alpha).  Profile
    scores carry the diagonal's offset change (+2 alpha, or (2 - G) alpha into
    a class-0 column), E is floored per class, and the running best pairs
    cell (r, j) (j even) with (r - 1, j + 1), which shares its offset, into one
    register per even class; the last row's odd columns are taken at the end
    (`tail`).  The carried state drops by rows * alpha at every period start.
    Returns the converted best."""
    assert G % 2 == 0 and T % G == 0
    B, m = Q.shape
    n = S.shape[1]
    f16 = np.float16
    a = alpha if (rows + G) * alpha < 1920 else 1920 // (rows + G)
    b = min(beta, 2048)
    nalpha, palpha, nu, rb, ng = f16(-a), f16(a), f16(a - b), f16(-rows * a), f16(-G * a)
    A = M.shape[0]
    Mx = np.zeros((A + 1, A + 1), np.int64)          # code A pads, scoring 0
    Mx[:A, :A] = M
    n_pad = ((n + chunk - 1) // chunk) * chunk + (chunk if extra_chunk else 0)
    m_pad = ((m + T - 1) // T) * T
    Qp = np.full((B, m_pad), A, np.int64)
    Qp[:, :m] = Q
    Sp = np.full((B, n_pad), A, np.int64)
    Sp[:, :n] = S
    bias = np.array([(2 - G) * a if j % G == 0 else 2 * a for j in range(m_pad)], np.int64)
    prof = [(Mx[Qp, Sp[:, r:r + 1]] + bias).astype(f16) for r in range(n_pad)]   # (B, m_pad)
    full = lambda v: np.full(B, f16(v), f16)
    best_true = np.zeros(B, f16)
    hb_out = f_out = None
    with np.errstate(over="ignore", invalid="ignore"):
        for k in range(m_pad // T):
            has_in = k > 0
            H = np.stack([full(((jj % G) - 1) * a) for jj in range(T)])
            E = np.stack([full((jj % G) * a) for jj in range(T)])    # true 0: H's floor
            fl = [full((1 + c) * a) for c in range(G)]
            z = full((G - 2) * a)
            bests = {c: full(0) for c in range(0, G, 2)}
            bests[0] = best_true.copy()
            hb_prev = full((G - 2) * a)
            new_hb, new_f = [], []
            for r in range(n_pad):
                if r and r % rows == 0:
                    H = (H + rb).astype(f16)
                    E = (E + rb).astype(f16)
                    fl = [(x + rb).astype(f16) for x in fl]
                    bests = {c: (x + rb).astype(f16) for c, x in bests.items()}
                    if has_in:
                        hb_prev = (hb_prev + rb).astype(f16)
                    else:
                        z = (z + rb).astype(f16)
                if has_in:
                    hdiag = hb_prev if r % chunk == 0 else hb_out[r - 1]
                    f = f_out[r]
                else:
                    hdiag, f = z, full(-a)
                h_even = None
                for jj in range(T):
                    j = k * T + jj
                    c = jj % G
                    hold = H[jj].copy()
                    h = np.maximum(np.maximum((hdiag + prof[r][:, j]).astype(f16), E[jj]), f)
                    t = (h + nu).astype(f16)
                    E[jj] = np.maximum(np.maximum(E[jj], t), fl[c])
                    f = np.maximum(f, t)
                    if c == G - 1:
                        f = (f + ng).astype(f16)
                    H[jj] = h
                    hdiag = hold
                    if jj % 2 == 0:
                        h_even = h
                    else:
                        bests[c - 1] = np.maximum(np.maximum(bests[c - 1], h_even), hdiag)
                new_hb.append(H[T - 1].copy())
                new_f.append(f.copy())
                fl = [(x + palpha).astype(f16) for x in fl]
                bests = {c: (x + palpha).astype(f16) for c, x in bests.items()}
                if not has_in:
                    z = (z + palpha).astype(f16)
                if has_in and r % chunk == chunk - 1:
                    hb_prev = hb_out[r]
            if tail:
                for jj in range(1, T, 2):
                    c = (jj - 1) % G
                    bests[c] = np.maximum(bests[c], H[jj])
            # bests[c] sits at offset fl[0] + (c - 1) alpha
            best_true = None
            for c, x in bests.items():
                v = (x - (fl[0] + f16((c - 1) * a)).astype(f16)).astype(f16)
                best_true = v if best_true is None else np.maximum(best_true, v)
            hb_out, f_out = new_hb, new_f
    assert not np.isnan(best_true).any()
    return best_true


def check_claim(orc, Q, S, M, alpha, beta, thr, tier, **kw):
    if tier == "f16":
        best = model_f16(Q, S, M, alpha, beta)
    elif tier == "frame":
        best = model_f16_frame(Q, S, M, alpha, beta, **kw)
    else:
        best = model_i16(Q, S, M, alpha, beta)
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


@pytest.mark.parametrize("thr", [1920, 700, 150])
@pytest.mark.parametrize("extra_chunk", [True, False])
def test_f16_row_frame_random(orc, thr, extra_chunk):
    """Lane-per-subject fp16 frame: subjects span several 32-row periods, the
    query several strips; penalties across the ceiling's range (alpha 0..200,
    every lane flagged past 53)."""
    rng = np.random.Generator(np.random.PCG64(thr + 11))
    for A, lo, hi in [(20, -4, 11), (4, -127, 127)]:
        M = rng.integers(lo, hi + 1, size=(A, A)).astype(np.int8)
        Q = rng.integers(0, A, size=(48, 21)).astype(np.uint8)
        S = rng.integers(0, A, size=(48, 76)).astype(np.uint8)
        for alpha, beta in [(0, 0), (2, 12), (5, 5), (28, 40), (29, 3000), (53, 60), (54, 54),
                            (57, 57), (200, 9000)]:
            check_claim(orc, Q, S, M, alpha, beta, lane_ceiling(thr, alpha), "frame",
                        extra_chunk=extra_chunk)


def test_f16_row_frame_two_classes(orc):
    """The same frame with two column classes (G = 2) also holds: the model is
    not tied to the kernel's G = 4 by accident."""
    rng = np.random.Generator(np.random.PCG64(12))
    M = rng.integers(-4, 12, size=(20, 20)).astype(np.int8)
    Q = rng.integers(0, 20, size=(48, 19)).astype(np.uint8)
    S = rng.integers(0, 20, size=(48, 70)).astype(np.uint8)
    for alpha, beta in [(2, 12), (5, 5), (50, 60)]:
        check_claim(orc, Q, S, M, alpha, beta, lane_ceiling(1920, alpha, G=2), "frame", G=2)


def test_f16_row_frame_scores_beyond_range(orc):
    """Copies and near-copies under a high diagonal: true scores from a few
    hundred to far past 2048 (and past the fp16 maximum); every lane at or
    above the ceiling must be flagged, every other exact."""
    rng = np.random.Generator(np.random.PCG64(5))
    A = 5
    M = np.full((A, A), -3, np.int8)
    np.fill_diagonal(M, 100)
    base = rng.integers(0, A, size=(40, 70)).astype(np.uint8)
    Q = base[:, :24].copy()
    S = base.copy()
    S[:, 30:54] = Q                     # the query planted mid-subject
    S[::3, 33::5] = (S[::3, 33::5] + 1) % A
    Q[1::4, :12] = rng.integers(0, A, size=(10, 12))
    for alpha in (1, 2, 20):
        check_claim(orc, Q, S, M, alpha, alpha + 10, lane_ceiling(1920, alpha), "frame")
    Qb = np.tile(np.arange(A, dtype=np.uint8), (3, 140))[:, :700]
    check_claim(orc, Qb[:, :40], Qb, M, 2, 12, lane_ceiling(1920, 2), "frame")


def test_frame_model_rejects_the_unshifted_ceiling(orc):
    """Negative control: with the ceiling of the unshifted form (1920) and
    alpha 20, an odd score of 1797 reached late in a 32-row period sits at an
    offset of up to 680, past 2048 where fp16 keeps only even integers, so
    unflagged lanes come out wrong; the frame ceiling (1200) flags them all."""
    rng = np.random.Generator(np.random.PCG64(9))
    A = 5
    M = np.full((A, A), -3, np.int8)
    np.fill_diagonal(M, 100)
    B = 64
    Q = rng.integers(0, A, size=(B, 19)).astype(np.uint8)
    S = rng.integers(0, A, size=(B, 70)).astype(np.uint8)
    for x in range(B):
        p = 20 + (x % 30)                   # the alignment ends at row p + 18
        S[x, p:p + 19] = Q[x]
        S[x, p + 3 + (x % 13)] = (S[x, p + 3 + (x % 13)] + 1) % A   # one mismatch: 1797
    check_claim(orc, Q, S, M, 20, 30, lane_ceiling(1920, 20), "frame")
    with pytest.raises(AssertionError):
        check_claim(orc, Q, S, M, 20, 30, 1920, "frame")


def test_frame_model_needs_the_last_row_tail(orc):
    """The running best takes the odd columns of row r at row r + 1, so the
    last row's odd columns need the closing step.  Queries of 16 residues
    planted at the very end of subjects of 40 (no padding rows): the best
    cell is the last row's last (odd) column.  Without the closing step the
    model must come out wrong."""
    rng = np.random.Generator(np.random.PCG64(17))
    A = 5
    M = np.full((A, A), -3, np.int8)
    np.fill_diagonal(M, 60)
    Q = rng.integers(0, A, size=(16, 16)).astype(np.uint8)
    S = rng.integers(0, A, size=(16, 40)).astype(np.uint8)
    S[:, 24:] = Q
    check_claim(orc, Q, S, M, 2, 12, lane_ceiling(1920, 2), "frame", extra_chunk=False)
    with pytest.raises(AssertionError):
        check_claim(orc, Q, S, M, 2, 12, lane_ceiling(1920, 2), "frame", extra_chunk=False,
                    tail=False)


def model_intra2_frame(Q, S, M, alpha, beta, T=4, lanes=64, rows=32, G=4, init_out_shift=True,
                       tail=True, grp=4):
    """Frame fp16 arithmetic of the packed wave-per-pair kernel, replayed step
    by step: `lanes` lanes of T query columns each (a pass covers lanes * T
    columns), lane l computing subject row t - l at step t, H and F of its last
    column handed to lane l+1 one step later, lane 0 fed from the previous
    pass's boundary (stored as true values) or from true 0, the last lane's
    outputs collected as true values for the next pass.  Cell (row, column jj
    of lane l) at step t sits at offset alpha * ((t mod rows) - l + (jj mod G)):
    E needs no decay, F decays by G alpha once per group of G columns, and the
    running best pairs (row, jj even) with (row - 1, jj + 1) into one register
    per even class, the last step's odd columns taken at the end (`tail`).
    Every carried value drops by rows * alpha at the end of each block of
    `rows` steps.  As in the kernel, a pass with outputs runs one step past
    its last block of `lanes` rows, and a pass without them rounds its steps
    up to a whole group of `grp`; the extra steps see only pad rows.
    Vectorised over pairs of equal shape (Q: (B, m), S: (B, n)).
    init_out_shift=False plants a wrong initial offset of the outputs handed
    on before step 0 (used by a negative control)."""
    assert G % 2 == 0 and T % G == 0
    B, m = Q.shape
    n = S.shape[1]
    f16 = np.float16
    a = min(alpha, 28)
    b = min(beta, 2048)
    nalpha, palpha, nu, rb, ng = f16(-a), f16(a), f16(a - b), f16(-rows * a), f16(-G * a)
    A = M.shape[0]
    Mx = np.zeros((A + 1, A + 1), np.int64)
    Mx[:A, :A] = M
    PW = lanes * T
    npass = (m + PW - 1) // PW
    Qp = np.full((B, npass * PW), A, np.int64)
    Qp[:, :m] = Q
    nblk = (n + lanes - 1) // lanes
    L = np.arange(lanes)
    cls = np.arange(T) % G
    bias = np.where(cls == 0, (2 - G) * a, 2 * a)                      # per lane column
    best_true = np.zeros(B, f16)
    bound_h = bound_f = None         # true values per row from the previous pass
    lanes_b = lambda v: np.broadcast_to(np.asarray(v, f16)[:, None], (lanes, B)).astype(f16).copy()
    with np.errstate(over="ignore", invalid="ignore"):
        for p in range(npass):
            has_in, has_out = p > 0, p + 1 < npass
            steps = nblk * lanes + lanes if has_out else (n + lanes - 1 + grp - 1) // grp * grp
            off0 = (-a * L).astype(np.int64)                          # (lanes,)
            H = np.stack([lanes_b(off0 + a * (cls[jj] - 1)) for jj in range(T)], axis=1)
            E = np.stack([lanes_b(off0 + a * cls[jj]) for jj in range(T)], axis=1)
            fl = [lanes_b(off0 + a * (1 + c)) for c in range(G)]
            bests = {c: lanes_b(off0 + a * c) for c in range(0, G, 2)}
            bests[0] = (best_true[None, :] + lanes_b(off0)).astype(f16)
            hb_prev = lanes_b(off0 + a * (G - 2))
            hout = lanes_b(off0 + a * (G - 2) if init_out_shift else off0 + a * (G - 1))
            fout = lanes_b(off0 - a)
            rowcode = np.full((lanes, B), A, np.int64)
            new_h = np.zeros((max(nblk, 1) * lanes, B), f16)
            new_f = np.zeros((max(nblk, 1) * lanes, B), f16)
            for t in range(steps):
                # lane 0 takes row t from the feeder, lane l the previous step's lane l-1
                fr = S[:, t] if t < n else np.full(B, A, np.int64)
                conv = a * (t % rows)
                if has_in and t < n:
                    fh = (bound_h[t] + f16(conv + a * (G - 1))).astype(f16)
                    ff = (bound_f[t] + f16(conv)).astype(f16)
                else:
                    fh = np.full(B, f16(conv + a * (G - 1)), f16)
                    ff = np.full(B, f16(conv), f16)
                rowcode = np.concatenate([fr[None, :], rowcode[:-1]])
                hin = np.concatenate([fh[None, :], hout[:-1]])
                fin = np.concatenate([ff[None, :], fout[:-1]])
                # one row per lane
                hdiag = hb_prev
                f = fin
                h_even = None
                for jj in range(T):
                    c = cls[jj]
                    col = p * PW + L * T + jj                          # (lanes,)
                    s = (Mx[Qp[:, col].T, rowcode] + bias[jj]).astype(f16)   # (lanes, B)
                    hold = H[:, jj].copy()
                    h = np.maximum(np.maximum((hdiag + s).astype(f16), E[:, jj]), f)
                    tt = (h + nu).astype(f16)
                    E[:, jj] = np.maximum(np.maximum(E[:, jj], tt), fl[c])
                    f = np.maximum(f, tt)
                    if c == G - 1:
                        f = (f + ng).astype(f16)
                    H[:, jj] = h
                    hdiag = hold
                    if jj % 2 == 0:
                        h_even = h
                    else:
                        bests[c - 1] = np.maximum(np.maximum(bests[c - 1], h_even), hold)
                hout = H[:, T - 1].copy()
                fout = f.copy()
                hb_prev = hin
                fl = [(x + palpha).astype(f16) for x in fl]
                bests = {c: (x + palpha).astype(f16) for c, x in bests.items()}
                # the last lane finished row t - (lanes - 1): store it as a true value
                r_done = t - (lanes - 1)
                if has_out and 0 <= r_done < new_h.shape[0]:
                    offw = a * ((t % rows) - (lanes - 1))
                    new_h[r_done] = (hout[-1] - f16(offw + a * (G - 1))).astype(f16)
                    new_f[r_done] = (fout[-1] - f16(offw)).astype(f16)
                if (t + 1) % rows == 0:
                    H = (H + rb).astype(f16)
                    E = (E + rb).astype(f16)
                    fl = [(x + rb).astype(f16) for x in fl]
                    bests = {c: (x + rb).astype(f16) for c, x in bests.items()}
                    hb_prev = (hb_prev + rb).astype(f16)
                    hout = (hout + rb).astype(f16)
                    fout = (fout + rb).astype(f16)
            if tail:
                for jj in range(1, T, 2):
                    bests[cls[jj] - 1] = np.maximum(bests[cls[jj] - 1], H[:, jj])
            oe = a * ((steps % rows) - L)                               # (lanes,)
            lane_best = None
            for c, x in bests.items():
                v = (x - lanes_b(oe + a * c)).astype(f16)
                lane_best = v if lane_best is None else np.maximum(lane_best, v)
            best_true = lane_best.max(axis=0)
            bound_h, bound_f = new_h, new_f
    assert not np.isnan(best_true).any()
    return best_true


def check_intra2(orc, Q, S, M, alpha, beta, thr, **kw):
    best = model_intra2_frame(Q, S, M, alpha, beta, **kw)
    for x in range(Q.shape[0]):
        exact = orc.sw_score(Q[x], S[x], M, alpha, beta)
        flagged = not (float(best[x]) < thr)
        assert flagged == (exact >= thr), (thr, exact, float(best[x]))
        if not flagged:
            assert int(best[x]) == exact, (thr, exact, float(best[x]))


@pytest.mark.parametrize("thr", [1920, 300, 20])
@pytest.mark.parametrize("T,G", [(4, 4), (2, 2)])
def test_intra2_row_frame_schedule(orc, thr, T, G):
    """Packed wave-per-pair schedule with 8 lanes of T columns (passes of 8T
    columns), column classes of G: one to three passes, subjects spanning
    several 32-step periods and several blocks of lanes, penalties across the
    alpha range."""
    rng = np.random.Generator(np.random.PCG64(thr + 5 + T))
    A = 20
    M = rng.integers(-4, 12, size=(A, A)).astype(np.int8)
    for m, n in [(5, 40), (8 * T, 70), (20 * T + 5, 90)]:
        Q = rng.integers(0, A, size=(12, m)).astype(np.uint8)
        S = rng.integers(0, A, size=(12, n)).astype(np.uint8)
        S[:3, 10:10 + min(m, 30)] = Q[:3, :min(m, 30)]        # some high scores
        for alpha, beta in [(2, 12), (1, 3), (28, 40)]:
            c = lane_ceiling(thr, alpha, G=G)
            check_intra2(orc, Q, S, M, alpha, beta, c, T=T, lanes=8, G=G)


def test_intra2_model_rejects_a_wrong_initial_offset(orc):
    """Negative control: H handed on before step 0 at one alpha above its
    offset gives a lane's first column a diagonal of true alpha on subject
    row 0.  Alignments planted to start there (row 0, lane 1's first column)
    must come out too high."""
    rng = np.random.Generator(np.random.PCG64(77))
    A = 20
    M = np.full((A, A), -3, np.int8)
    np.fill_diagonal(M, 40)
    Q = rng.integers(0, A, size=(12, 20)).astype(np.uint8)
    S = rng.integers(0, A, size=(12, 50)).astype(np.uint8)
    S[:, :16] = Q[:, 4:20]
    check_intra2(orc, Q, S, M, 2, 12, 1848, T=4, lanes=8)
    with pytest.raises(AssertionError):
        check_intra2(orc, Q, S, M, 2, 12, 1848, T=4, lanes=8, init_out_shift=False)


def test_intra2_model_needs_the_last_step_tail(orc):
    """The running best takes a lane's odd columns of row r at row r + 1; the
    last lane meets its last real row at the last step unless the pass rounds
    its steps up with pad rows.  Subjects of 49 rows (49 + 8 - 1 steps, a
    whole number of groups, so no pad step) with queries planted at their
    end (best cell in the last lane's last column, last row): without the
    closing step the model must come out wrong."""
    rng = np.random.Generator(np.random.PCG64(19))
    A = 5
    M = np.full((A, A), -3, np.int8)
    np.fill_diagonal(M, 40)
    Q = rng.integers(0, A, size=(8, 32)).astype(np.uint8)       # 8 lanes x 4 columns: one pass
    S = rng.integers(0, A, size=(8, 49)).astype(np.uint8)
    S[:, 17:] = Q
    check_intra2(orc, Q, S, M, 2, 12, 1848, T=4, lanes=8)
    with pytest.raises(AssertionError):
        check_intra2(orc, Q, S, M, 2, 12, 1848, T=4, lanes=8, tail=False)
