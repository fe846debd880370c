"""Databases larger than device memory: an on-disk index searched chunk by
chunk (section III's offline index and chunked loading), against the same
database opened whole and against the oracle.

The database has 1,200,000 subjects (mean 30 residues) plus 40 subjects
longer than the lane-per-subject groups take, dealt round-robin in length
order into 7 chunks of up to 6 M residues: each holds about 171,000 subjects
of every length, enough for lane-per-subject groups, and a few long ones.  A
memory budget of 40 MiB forces streaming through two device slots; the
default budget keeps every chunk resident.  A second index, whose subjects
are long next to its chunks, is cut into consecutive runs of the length
order instead: every chunk runs wave-per-pair.
"""
import numpy as np
import pytest

import oracle
import synthdata as sd

pytestmark = pytest.mark.gpu

K = 50


@pytest.fixture(scope="module")
def data(tmp_path_factory):
    import paper_1404_4152_amd as swmi
    swmi.lib()
    rng = np.random.Generator(np.random.PCG64(515))
    res, off = sd.make_db(1_200_000, 30, 5, 200, seed=515)
    extra = [sd.random_residues(rng, int(x)) for x in rng.integers(8200, 12000, size=40)]
    seqs = [res[off[i]:off[i + 1]] for i in range(len(off) - 1)] + extra
    order = rng.permutation(len(seqs))          # the long ones scattered through the database
    res, off = sd.pack_sequences([seqs[i] for i in order])
    queries = [sd.random_residues(rng, n) for n in (60, 233, 701)]
    # a near-copy of query 2 inside the database: a score past the fp16 ceiling
    res, off = sd.rebuild_db(res, off, {12345: sd.mutate(rng, queries[2], 0.95)})
    path = tmp_path_factory.mktemp("index") / "db.swx"
    swmi.sw_index_write(str(path), res, off, 20, 6_000_000)
    return swmi, res, off, queries, str(path)


@pytest.fixture(scope="module")
def whole(data):
    swmi, res, off, queries, path = data
    M = sd.blosum_style_matrix()
    db = swmi.Database(res, off, 20)
    try:
        ts, ti, al = db.search_batch(queries, M, 2, 12, K, all_scores=True)
    finally:
        db.close()
    return ts, ti, al


@pytest.mark.parametrize("budget", [40 << 20, 0])
def test_index_equals_whole_database(data, whole, budget):
    swmi, res, off, queries, path = data
    M = sd.blosum_style_matrix()
    print(f"index search, memory budget {budget}", flush=True)
    ix = swmi.Index(path, memory_budget=budget)
    try:
        assert ix.n == len(off) - 1
        ts, ti, al = ix.search_batch(queries, M, 2, 12, K, all_scores=True)
        st = ix.stats()
        # twice: the slots already hold chunks from the first call
        ts2, ti2 = ix.search_batch(queries, M, 2, 12, K)
    finally:
        ix.close()
    assert st["chunks"] >= 3
    assert st["resident"] == (1 if budget == 0 else 0)
    if budget:
        assert st["bytes_loaded"] > 0
    assert st["cells"] == sum(len(q) for q in queries) * int(off[-1])
    wts, wti, wal = whole
    assert np.array_equal(al, wal)
    assert np.array_equal(ts, wts) and np.array_equal(ti, wti)
    assert np.array_equal(ts2, wts) and np.array_equal(ti2, wti)
    assert al[2, 12345] >= 1848


def test_index_against_oracle(data):
    swmi, res, off, queries, path = data
    M = sd.blosum_style_matrix()
    orc = oracle.load()
    ix = swmi.Index(path, memory_budget=40 << 20)
    try:
        ts, ti, al = ix.search_batch(queries[:2], M, 2, 12, K, all_scores=True)
    finally:
        ix.close()
    for x, q in enumerate(queries[:2]):
        print(f"oracle, query {x} ({len(q)} residues)", flush=True)
        exp = orc.search(q, res, off, M, 2, 12)
        bad = np.flatnonzero(al[x] != exp)
        assert bad.size == 0, (x, bad[:5].tolist(), al[x][bad[:5]].tolist(), exp[bad[:5]].tolist())
        es, ei = oracle.topk(exp, K)
        assert np.array_equal(ts[x], es) and np.array_equal(ti[x], ei)


def test_index_ties_across_chunks(data):
    """A one-residue query scores every subject holding its residue the same:
    the merged top-k must take the lowest database indices among equal scores,
    whichever chunk holds them."""
    swmi, res, off, queries, path = data
    M = sd.blosum_style_matrix()
    q = np.array([17], np.uint8)
    ix = swmi.Index(path, memory_budget=40 << 20)
    try:
        ts, ti = ix.search_batch([q], M, 2, 12, 300)
    finally:
        ix.close()
    orc = oracle.load()
    exp = orc.search(q, res, off, M, 2, 12)
    es, ei = oracle.topk(exp, 300)
    assert np.array_equal(ts[0], es) and np.array_equal(ti[0], ei)


def test_index_budget_too_small(data):
    swmi, res, off, queries, path = data
    with pytest.raises(swmi.SwError) as e:
        swmi.Index(path, memory_budget=10 << 20)
    assert e.value.code == swmi.SW_ENOMEM and "budget" in str(e.value)


def test_index_length_runs_streamed(tmp_path):
    """Subjects of up to 4,530 residues in chunks of 15,000: too long to deal
    round-robin (more than a quarter of a chunk), so the chunks are
    consecutive runs of the length order (the file says which), each too small
    for lane-per-subject groups; streamed under a small budget, the results
    equal the whole database's."""
    import paper_1404_4152_amd as swmi
    rng = np.random.Generator(np.random.PCG64(77))
    res, off = sd.make_db(3000, 300, 0, 9000, seed=77)
    path = tmp_path / "runs.swx"
    swmi.sw_index_write(str(path), res, off, 20, 15_000)
    assert int(np.frombuffer(path.read_bytes()[:72], np.int64, 1, 48)[0]) == 0   # header: layout 0
    M = sd.blosum_style_matrix()
    queries = [sd.random_residues(rng, n) for n in (50, 300, 1100)]
    db = swmi.Database(res, off, 20)
    try:
        wts, wti, wal = db.search_batch(queries, M, 2, 12, 20, all_scores=True)
    finally:
        db.close()
    print("length-run index, streamed", flush=True)
    ix = swmi.Index(str(path), memory_budget=256 << 10)
    try:
        ts, ti, al = ix.search_batch(queries, M, 2, 12, 20, all_scores=True)
        st = ix.stats()
    finally:
        ix.close()
    assert st["resident"] == 0 and st["chunks"] > 20
    assert np.array_equal(al, wal)
    assert np.array_equal(ts, wts) and np.array_equal(ti, wti)


@pytest.mark.parametrize("seed", range(10))
def test_index_random_configs(tmp_path, seed):
    """Seeded draws of database size, lengths, chunk size (dealt or in runs)
    and memory budget (resident or streamed): the index's scores and top-k
    equal the whole database's."""
    import paper_1404_4152_amd as swmi
    rng = np.random.Generator(np.random.PCG64(31_000 + seed))
    n = int(rng.choice([50, 2000, 20000]))
    hi = int(rng.choice([40, 400, 3000]))
    lens = rng.integers(0, hi + 1, size=n)
    res, off = sd.pack_sequences([sd.random_residues(rng, int(L)) for L in lens])
    total = int(off[-1])
    chunk = int(max(1, total // int(rng.choice([1, 3, 7, 40]))))
    path = tmp_path / "r.swx"
    swmi.sw_index_write(str(path), res, off, 20, chunk)
    layout = int(np.frombuffer(path.read_bytes()[:72], np.int64, 1, 48)[0])
    M = sd.blosum_style_matrix()
    qs = [sd.random_residues(rng, int(L)) for L in rng.integers(1, 900, size=2)]
    k = int(rng.choice([1, 10, 64]))
    budget = int(rng.choice([0, 1 << 20, 8 << 20]))
    print(f"index seed {seed}: n {n} hi {hi} chunk {chunk} layout {layout} budget {budget} k {k}", flush=True)
    db = swmi.Database(res, off, 20)
    try:
        wts, wti, wal = db.search_batch(qs, M, 2, 12, k, all_scores=True)
    finally:
        db.close()
    try:
        ix = swmi.Index(str(path), memory_budget=budget)
    except swmi.SwError as e:
        # a budget below two of the largest chunk is refused, and says so
        assert e.code == swmi.SW_ENOMEM and "budget" in str(e) and budget > 0
        return
    try:
        ts, ti, al = ix.search_batch(qs, M, 2, 12, k, all_scores=True)
    finally:
        ix.close()
    assert np.array_equal(al, wal)
    assert np.array_equal(ts, wts) and np.array_equal(ti, wti)
