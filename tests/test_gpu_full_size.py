"""GPU parity at the benchmark's full sizes, in the launch configuration that
bench.py times, on outputs the oracle computes one by one, plus properties that
hold at any size.

plain_scale: 2,000,000 subjects (0.70 G residues) and the 144-, 1,000- and
5,478-residue queries of that workload, fp16 tier, strip 32 with 4 and with 8
waves per workgroup (the plans the autotuner picks on this database).  Every
query runs through the lane-per-subject kernel, the long list overlapped on the
second stream and the top-k, exactly as in the timed steps.

batched: 512 queries x 500,000 subjects in one launch, replayed from the
captured HIP graph.

long_tail: 20,000 subjects of 5,000-35,000 residues, all wave-per-pair.

serving: 5,000,000 subjects resident under the server; each request's top-k
is recomputed by the oracle and compared with a plain search of the same
database once the server has stopped.

Checked on every output: scores >= 0, empty subjects score 0, and the
library's top-k equals the (score desc, index asc) top-k of the full vector.
Checked against the oracle: the top hits, the longest subjects (the long list)
and a random sample of subjects.
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


def top_of(scores, k):
    """(score desc, index asc) top-k of one score vector, in O(n)."""
    k = min(k, len(scores))
    if k == 0:
        return np.zeros(0, np.int32), np.zeros(0, np.int64)
    kth = np.partition(scores, len(scores) - k)[len(scores) - k]
    cand = np.flatnonzero(scores >= kth)
    order = np.lexsort((cand, -scores[cand].astype(np.int64)))[:k]
    idx = cand[order]
    return scores[idx], idx.astype(np.int64)


def sample_ids(rng, lens, extra, n_random, n_long):
    n = len(lens)
    longest = np.argsort(-lens, kind="stable")[:n_long]
    rand = rng.choice(n, size=min(n_random, n), replace=False)
    return np.unique(np.concatenate([rand, longest, np.asarray(extra, np.int64)]))


def check_vector(orc, q, res, off, M, alpha, beta, got, ts, ti, rng, what, n_random, n_long):
    lens = np.diff(off)
    assert got.shape == (len(lens),)
    assert (got >= 0).all(), what
    assert (got[lens == 0] == 0).all(), what
    es, ei = top_of(got, len(ts))
    assert np.array_equal(ts, es) and np.array_equal(ti, ei), (what, ts[:5], es[:5], ti[:5], ei[:5])
    which = sample_ids(rng, lens, ti, n_random, n_long)
    exp = orc.search_subset(q, res, off, which, M, alpha, beta)
    bad = np.flatnonzero(got[which] != exp)
    assert bad.size == 0, (f"{what}: {bad.size} of {len(which)} sampled scores differ, first ids "
                           f"{which[bad[:5]].tolist()}: got {got[which[bad[:5]]].tolist()} "
                           f"expected {exp[bad[:5]].tolist()}")


@pytest.fixture(scope="module")
def plain_db(swmi):
    w = sd.WORKLOADS["plain_scale"]
    res, off = w.db()
    db = swmi.Database(res, off, 20)
    yield w, res, off, db
    db.close()


@pytest.mark.parametrize("waves", [4, 8])
def test_plain_scale_full_size_sampled(swmi, orc, plain_db, waves):
    w, res, off, db = plain_db
    M = w.matrix()
    qs = w.queries()
    rng = np.random.Generator(np.random.PCG64(2024 + waves))
    db.set_opts(tier=1, strip=32, waves=waves)
    for qi in (0, 9, 19):
        q = qs[qi]
        print(f"plain_scale full size: plan 1/32/{waves}, query {qi} ({len(q)} residues)", flush=True)
        ts, ti = db.topk(q, M, w.alpha, w.beta, 10)
        st = db.stats()
        assert st["tier"] == 1 and st["strip"] == 32 and st["waves"] == waves
        assert st["inter_cells"] > 0 and st["intra_pairs"] > 0
        got = db.search(q, M, w.alpha, w.beta)
        check_vector(orc, q, res, off, M, w.alpha, w.beta, got, ts, ti, rng,
                     f"plain_scale q{qi} waves {waves}", n_random=3000, n_long=150)
    db.set_opts(reset=True)


def test_batched_full_size_sampled(swmi, orc):
    w = sd.WORKLOADS["batched"]
    res, off = w.db()
    M = w.matrix()
    qs = w.queries()
    assert len(qs) == 512
    rng = np.random.Generator(np.random.PCG64(77))
    db = swmi.Database(res, off, 20)
    try:
        print("batched full size: capture", flush=True)
        db.search_batch(qs, M, w.alpha, w.beta, 10)
        print("batched full size: replay with every score", flush=True)
        ts, ti, al = db.search_batch(qs, M, w.alpha, w.beta, 10, all_scores=True)
        assert db.stats()["graphed"] == 1
        n = len(off) - 1
        al = al.reshape(len(qs), n)
        for x in range(len(qs)):
            es, ei = top_of(al[x], 10)
            assert np.array_equal(ts[x], es) and np.array_equal(ti[x], ei), f"batched top-k q{x}"
        assert (al >= 0).all()
        assert (al[:, np.diff(off) == 0] == 0).all()
        for x in rng.choice(len(qs), size=8, replace=False):
            check_vector(orc, qs[x], res, off, M, w.alpha, w.beta, al[x], ts[x], ti[x], rng,
                         f"batched q{x}", n_random=500, n_long=20)
    finally:
        db.close()


def test_long_tail_full_size_sampled(swmi, orc):
    """long_tail: 20,000 subjects of 5,000-35,000 residues (every one past the
    8,192-residue group limit, so all wave-per-pair), queries of 1,000 and
    5,000 residues in the fp16 plan (packed kernel, several passes)."""
    w = sd.WORKLOADS["long_tail"]
    res, off = w.db()
    M = w.matrix()
    qs = w.queries()
    rng = np.random.Generator(np.random.PCG64(31))
    db = swmi.Database(res, off, 20)
    try:
        for qi in (0, len(qs) - 1):
            q = qs[qi]
            print(f"long_tail full size: query {qi} ({len(q)} residues)", flush=True)
            ts, ti = db.topk(q, M, w.alpha, w.beta, 10)
            st = db.stats()
            assert st["intra_pairs"] == len(off) - 1 and st["inter_cells"] == 0
            got = db.search(q, M, w.alpha, w.beta)
            check_vector(orc, q, res, off, M, w.alpha, w.beta, got, ts, ti, rng,
                         f"long_tail q{qi}", n_random=60, n_long=10)
    finally:
        db.close()


def test_served_full_size_sampled(swmi, orc):
    """serving: 5,000,000 subjects (1.75 G residues) resident; requests of the
    serving query mix submitted together, so passes mix requests at different
    scan positions.  Each request's top-k is recomputed by the oracle, and
    once the server is stopped it must equal a plain search of the same
    database (verified elsewhere against the oracle)."""
    w = sd.WORKLOADS["serving"]
    res, off = w.db()
    M = w.matrix()
    qs = sd.serving_queries(6)
    k = 10
    db = swmi.Database(res, off, 20)
    try:
        srv = swmi.sw_server_start(db.h, memory_budget=8 << 30, max_active=64)
        try:
            print("served full size: submit", [len(q) for q in qs], flush=True)
            tickets = [swmi.sw_server_submit(srv, q, M, w.alpha, w.beta, k) for q in qs]
            results = [swmi.sw_server_wait(srv, t, k) for t in tickets]
        finally:
            swmi.sw_server_stop(srv)
        for x, (q, (ts, ti, st)) in enumerate(zip(qs, results)):
            assert st["passes"] >= 1
            exp = orc.search_subset(q, res, off, ti, M, w.alpha, w.beta)
            assert np.array_equal(ts, exp), f"served q{x}: top-k scores differ from the oracle"
            ps, pi = db.topk(q, M, w.alpha, w.beta, k)
            assert np.array_equal(ts, ps) and np.array_equal(ti, pi), f"served q{x} != plain search"
    finally:
        db.close()
