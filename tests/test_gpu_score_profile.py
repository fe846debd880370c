"""GPU parity of the score-profile variant of the lane-per-subject kernel
(section III.B.3), selected with sw_search_opts.profile = SW_PROFILE_SCORE,
bit-exact against the oracle through the C ABI.

Covered: query lengths around the strip of 32 and over many strips (ragged
last strip, columns past the query scoring through the pad letter), zero-
length subjects and a ragged last group, alphabets of 3, 20 and 23 letters
(the kernel's limit; 24 falls back to the pair profile), asymmetric matrices
(the table row of a subject-residue pair is the matrix column), alpha from 0
to the fp16 frame's limit, forced overflow recompute, planted homologs above
the fp16 ceiling, and a batch of queries with different lengths in one
launch and its graph replays (the letter-pair table is rebuilt when a
workgroup moves to another query).
"""
import numpy as np
import pytest

import oracle
import synthdata as sd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def swmi():
    import paper_1404_4152_amd as p
    p.lib()
    return p


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


def random_db(rng, n, A, lo, hi, zero_every=0):
    lens = rng.integers(lo, hi + 1, size=n)
    if zero_every:
        lens[::zero_every] = 0
    return sd.pack_sequences([rng.integers(0, A, size=int(L)).astype(np.uint8) for L in lens])


def expect_equal(got, exp, what):
    bad = np.flatnonzero(np.asarray(got) != np.asarray(exp))
    assert bad.size == 0, (f"{what}: {bad.size} mismatches, first at {bad[:5].tolist()}: "
                           f"got {np.asarray(got)[bad[:5]].tolist()} expected {np.asarray(exp)[bad[:5]].tolist()}")


@pytest.mark.parametrize("A", [3, 20, 23])
def test_score_profile_random(swmi, orc, A):
    rng = np.random.Generator(np.random.PCG64(31 + A))
    M = sd.random_matrix(rng, A) if A != 20 else sd.blosum_style_matrix()
    res, off = random_db(rng, 128 * 4 * 3 + 59, A, 1, 300, zero_every=47)
    db = swmi.Database(res, off, A, long_threshold=-1)
    try:
        db.set_opts(tier=1, strip=32, waves=4, profile=1)
        for L in [1, 5, 31, 32, 33, 64, 95, 257, 700]:
            q = rng.integers(0, A, size=L).astype(np.uint8)
            for alpha, beta in [(2, 12), (0, 5), (1, 1), (28, 40)]:
                print(f"A={A} qlen={L} alpha={alpha} beta={beta}", flush=True)
                got = db.search(q, M, alpha, beta)
                st = db.stats()
                assert st["profile"] == 1 and st["tier"] == 1 and st["inter_cells"] > 0
                expect_equal(got, orc.search(q, res, off, M, alpha, beta),
                             f"A {A} qlen {L} alpha {alpha} beta {beta}")
    finally:
        db.close()


def test_score_profile_asymmetric_and_overflow(swmi, orc):
    """An asymmetric matrix, a forced low threshold (many lanes flagged and
    recomputed in int32) and planted near-copies above the fp16 ceiling."""
    rng = np.random.Generator(np.random.PCG64(4711))
    A = 20
    M = sd.random_matrix(rng, A, lo=-5, hi=11)
    assert not (M == M.T).all()
    res, off = random_db(rng, 1500, A, 10, 400, zero_every=61)
    q = rng.integers(0, A, size=420).astype(np.uint8)
    res, off = sd.rebuild_db(res, off, {3: sd.mutate(rng, q, 0.95), 700: q.copy()})
    db = swmi.Database(res, off, A, long_threshold=-1)
    try:
        exp = orc.search(q, res, off, M, 2, 12)
        assert exp[700] >= 1848
        db.set_opts(tier=1, strip=32, waves=4, profile=1)
        expect_equal(db.search(q, M, 2, 12), exp, "planted")
        assert db.stats()["recomputed_pairs"] >= 1
        db.set_opts(tier=1, strip=32, waves=4, profile=1, sat_threshold=30)
        expect_equal(db.search(q, M, 2, 12), exp, "forced threshold")
        assert db.stats()["recomputed_pairs"] > 100
    finally:
        db.close()


def test_score_profile_batch_and_graph(swmi, orc):
    """Queries of different lengths in one launch (a workgroup meets several
    queries and rebuilds its table), captured once and replayed."""
    rng = np.random.Generator(np.random.PCG64(99))
    A = 20
    M = sd.blosum_style_matrix()
    res, off = random_db(rng, 128 * 4 * 4 + 3, A, 0, 250, zero_every=29)
    db = swmi.Database(res, off, A, long_threshold=-1)
    try:
        db.set_opts(tier=1, strip=32, waves=4, profile=1)
        for rep in range(3):
            qs = [sd.random_residues(rng, L) for L in (17, 300, 64, 129)]
            print(f"batch rep {rep}", flush=True)
            ts, ti, al = db.search_batch(qs, M, 2, 12, 7, all_scores=True)
            assert db.stats()["profile"] == 1
            for x, q in enumerate(qs):
                exp = orc.search(q, res, off, M, 2, 12)
                expect_equal(al[x], exp, f"rep {rep} q{x}")
                es, ei = oracle.topk(exp, 7)
                assert np.array_equal(ts[x], es) and np.array_equal(ti[x], ei)
    finally:
        db.close()


def test_score_profile_falls_back(swmi, orc):
    """Plans the variant does not cover run the pair profile and say so."""
    rng = np.random.Generator(np.random.PCG64(5))
    res, off = random_db(rng, 700, 24, 1, 200)
    M = sd.random_matrix(rng, 24)
    q = rng.integers(0, 24, size=90).astype(np.uint8)
    db = swmi.Database(res, off, 24, long_threshold=-1)
    try:
        db.set_opts(tier=1, strip=32, waves=4, profile=1)
        expect_equal(db.search(q, M, 2, 12), orc.search(q, res, off, M, 2, 12), "A = 24")
        assert db.stats()["profile"] == 0
    finally:
        db.close()
    res, off = random_db(rng, 700, 20, 1, 200)
    M = sd.blosum_style_matrix()
    q = sd.random_residues(rng, 90)
    db = swmi.Database(res, off, 20, long_threshold=-1)
    try:
        db.set_opts(tier=1, strip=16, waves=4, profile=1)
        expect_equal(db.search(q, M, 2, 12), orc.search(q, res, off, M, 2, 12), "strip 16")
        assert db.stats()["profile"] == 0
        db.set_opts(profile=1)   # the planner takes the int16 tier above alpha 28
        expect_equal(db.search(q, M, 40, 60), orc.search(q, res, off, M, 40, 60), "alpha 40")
        assert db.stats()["profile"] == 0 and db.stats()["tier"] == 2
    finally:
        db.close()
