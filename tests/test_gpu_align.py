"""GPU parity of sw_db_align (alignment with traceback) against the oracle's
oracle_sw_align, alignment by alignment: score, begin and end positions and
every run must be identical.  The oracle itself is pinned by rescoring, the
end-cell rule against the cubic recurrence and hand-worked tie cases
(tests/pins.py); the GPU path shares no code with it."""
import numpy as np
import pytest

import oracle
import pins
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


def check_all(orc, got, q, res, off, ids, M, alpha, beta, what):
    assert len(got) == len(ids)
    for k, (g, i) in enumerate(zip(got, ids)):
        exp = orc.sw_align(q, res[off[i]:off[i + 1]], M, alpha, beta)
        assert g == exp, f"{what}: id {i} (pair {k}): got {g}, expected {exp}"


@pytest.mark.parametrize("qlen", [1, 37, 1024, 1025, 2500, 4000, 4100, 6100, 6200])
def test_random_db_align(swmi, orc, qlen):
    """Subjects of 0..1,500 residues (some empty), a query copy planted in
    some.  The query lengths reach every forward kernel: one wave per pair
    for a single pass (1, 37) and for passes that do not fit a workgroup
    (6,200: seven passes of 1,024 columns, one after another); one wave per
    pass, pipelined, at 4 columns per lane (1,024 to 4,000: 4 to 16 passes,
    16 being the most waves a workgroup takes) and at 8 (4,100 and 6,100: 9
    and 12 passes, 12 filling the LDS)."""
    rng = np.random.Generator(np.random.PCG64(500 + qlen))
    A = 20
    M = sd.blosum_style_matrix()
    q = sd.random_residues(rng, qlen)
    seqs = [sd.random_residues(rng, int(L)) for L in rng.integers(0, 1500, size=120)]
    seqs[3] = np.zeros(0, np.uint8)
    seqs[7] = np.concatenate([sd.random_residues(rng, 40), q[: min(qlen, 300)], sd.random_residues(rng, 9)])
    res, off = sd.pack_sequences(seqs)
    db = swmi.Database(res, off, A)
    try:
        ids = list(range(len(seqs))) + [7, 3]          # repeats allowed
        print(f"align qlen={qlen} pairs={len(ids)}", flush=True)
        got = db.align(q, M, 2, 12, ids)
        check_all(orc, got, q, res, off, ids, M, 2, 12, f"qlen {qlen}")
        scores = db.search(q, M, 2, 12)
        assert [g["score"] for g in got] == [int(scores[i]) for i in ids]
    finally:
        db.close()


@pytest.mark.parametrize("alpha,beta", [(2, 2), (0, 0), (1, 3), (3, 3)])
def test_tie_heavy_align(swmi, orc, alpha, beta):
    """Alphabet of 3 with repeats, equal scores everywhere and alpha = beta:
    most cells tie, so every tie rule of the traceback decides."""
    rng = np.random.Generator(np.random.PCG64(77 + alpha + 7 * beta))
    A = 3
    M = np.array([[4, -2, -2], [-2, 4, -2], [-2, -2, 4]], np.int8)
    q = rng.integers(0, A, size=90).astype(np.uint8)
    seqs = [rng.integers(0, A, size=int(L)).astype(np.uint8) for L in rng.integers(1, 200, size=40)]
    seqs[0] = np.tile(q[:10], 6)
    res, off = sd.pack_sequences(seqs)
    db = swmi.Database(res, off, A)
    try:
        print(f"tie-heavy alpha={alpha} beta={beta}", flush=True)
        ids = list(range(len(seqs)))
        check_all(orc, db.align(q, M, alpha, beta, ids), q, res, off, ids, M, alpha, beta,
                  f"ties {alpha}/{beta}")
    finally:
        db.close()


def test_golden_alignments_on_gpu(swmi):
    """The hand-worked tie cases of tests/golden/align_examples.txt."""
    for name, q, s, M, a, b, exp in pins.load_golden_align():
        res, off = sd.pack_sequences([s])
        db = swmi.Database(res, off, M.shape[0])
        try:
            print(f"golden {name}", flush=True)
            got = db.align(q, M, a, b, [0])[0]
            assert got == exp, (name, got, exp)
        finally:
            db.close()


def test_top_hits_long_subjects(swmi, orc):
    """long_tail database (subjects of 5,000-35,000): the top-6 hits of a
    5,000-residue query, about 1 GB of traceback bytes, so the pairs run in
    more than one batch."""
    w = sd.WORKLOADS["long_tail"]
    res, off = w.db()
    M = w.matrix()
    q = w.queries()[-1]
    db = swmi.Database(res, off, 20)
    try:
        ts, ti = db.topk(q, M, w.alpha, w.beta, 6)
        lens = np.diff(off)[ti]
        print(f"top hits of {len(q)} residues: subject lengths {lens.tolist()}", flush=True)
        got = db.align(q, M, w.alpha, w.beta, ti)
        assert [g["score"] for g in got] == ts.tolist()
        check_all(orc, got, q, res, off, ti, M, w.alpha, w.beta, "long_tail top hits")
    finally:
        db.close()


def test_align_rejects_bad_arguments(swmi):
    rng = np.random.Generator(np.random.PCG64(3))
    res, off = sd.pack_sequences([sd.random_residues(rng, 50) for _ in range(4)])
    db = swmi.Database(res, off, 20)
    M = sd.blosum_style_matrix()
    try:
        with pytest.raises(swmi.SwError):
            db.align(sd.random_residues(rng, 10), M, 2, 12, [4])      # id out of range
        with pytest.raises(swmi.SwError):
            db.align(sd.random_residues(rng, 10), M, 3, 2, [0])       # beta < alpha
        assert db.align(sd.random_residues(rng, 10), M, 2, 12, []) == []
    finally:
        db.close()
