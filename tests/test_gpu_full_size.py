"""GPU parity at the benchmark's full sizes, in the launch configuration that
bench.py times, against the oracle's own full results.

tests/golden/full_size.json holds, per query, the SHA-256 of the oracle's
full int32 score vector (database order) and the oracle's top-10 (score
descending, index ascending); tests/golden/make_full_size.py wrote it by
calling only oracle/.  Each test here computes the same vector on the GPU and
requires the same digest and the same top-10, so every score of every
subject is compared, not a sample.  When a digest differs, the subjects that
differ are named from a sampled oracle comparison (the top hits, the longest
subjects and a random sample) before the test fails.

plain_scale: 2,000,000 subjects (0.70 G residues, length-sorted, a planted
family of homologs per query), all 20 queries (144..5,478 residues), fp16
tier, strip 32 with 4 and with 8 waves per workgroup (the plans the
autotuner picks on this database).  Every query runs through the
lane-per-subject kernel, the long list and the top-k, as in the timed steps.

batched: 512 queries x 500,000 subjects in one launch replayed from the
captured HIP graph; a seeded sample of 16 of the 512 score rows is compared
in full, and every row's top-k against the top-k of its own row.

long_tail: 20,000 subjects of 5,000-35,000 residues (all wave-per-pair), all
8 queries, each with an 85%-identity homolog embedded in one subject (scores
above the fp16 ceiling, recomputed exactly in int32).

serving: 5,000,000 subjects resident under the server; 6 requests of the
serving query mix submitted together.  Each served top-10 must equal the
oracle's top-10 over the whole database, and a plain search of each query
must give the oracle's full score vector.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import synthdata as sd

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size.json")


@pytest.fixture(scope="module")
def swmi():
    import paper_1404_4152_amd as p
    p.lib()
    return p


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def vector_sha256(scores):
    return hashlib.sha256(np.ascontiguousarray(scores, dtype="<i4").tobytes()).hexdigest()


def workload_record(golden, name, res, off, M, w):
    """The stored record of one workload, after checking that it was written
    for exactly these inputs."""
    rec = golden.get(name)
    assert rec is not None, f"{name}: no oracle records (tests/golden/make_full_size.py writes them)"
    assert rec["db_sha256"] == sd.sha256(res, off), f"{name}: database differs from the record's"
    assert rec["matrix_sha256"] == sd.sha256(M), f"{name}: matrix differs from the record's"
    assert (rec["alpha"], rec["beta"]) == (w.alpha, w.beta)
    return rec


def query_record(rec, name, i, q):
    """The stored record of query i (tests/test_golden_complete.py checks on
    the CPU that every record is there)."""
    e = rec["queries"].get(str(i))
    assert e is not None, f"{name} q{i}: no oracle record"
    assert e["query_sha256"] == sd.sha256(q) and e["qlen"] == len(q), f"{name} q{i}: query differs"
    return e


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


def name_differences(orc, q, res, off, M, alpha, beta, got, extra, rng, n_random=2000, n_long=100):
    """Subjects whose GPU score differs from the oracle's, among the top hits,
    the longest subjects and a random sample (for the failure message)."""
    lens = np.diff(off)
    n = len(lens)
    longest = np.argsort(-lens, kind="stable")[:n_long]
    rand = rng.choice(n, size=min(n_random, n), replace=False)
    which = np.unique(np.concatenate([rand, longest, np.asarray(extra, np.int64)]))
    exp = orc.search_subset(q, res, off, which, M, alpha, beta)
    bad = np.flatnonzero(got[which] != exp)
    return (f"{bad.size} of {len(which)} sampled scores differ; first ids {which[bad[:5]].tolist()}: "
            f"got {got[which[bad[:5]]].tolist()} expected {exp[bad[:5]].tolist()}")


def check_full(orc, e, q, res, off, M, w, got, ts, ti, what, seed):
    """Full vector digest, oracle top-10, plus the properties any output has."""
    lens = np.diff(off)
    assert got.shape == (len(lens),), what
    assert (got >= 0).all(), what
    assert (got[lens == 0] == 0).all(), what
    k = len(e["top_scores"])
    ok_top = (np.array_equal(ts[:k], np.asarray(e["top_scores"], np.int32)) and
              np.array_equal(ti[:k], np.asarray(e["top_idx"], np.int64)))
    ok_vec = vector_sha256(got) == e["scores_sha256"]
    if not (ok_top and ok_vec):
        rng = np.random.Generator(np.random.PCG64(seed))
        msg = name_differences(orc, q, res, off, M, w.alpha, w.beta, got,
                               np.concatenate([ti, np.asarray(e["top_idx"])]), rng)
        pytest.fail(f"{what}: full vector {'matches' if ok_vec else 'differs'}, top-{k} "
                    f"{'matches' if ok_top else 'differs'} (got {ts[:k].tolist()} / {ti[:k].tolist()}, "
                    f"oracle {e['top_scores']} / {e['top_idx']}); {msg}")


@pytest.fixture(scope="module")
def plain_db(swmi, golden):
    w = sd.WORKLOADS["plain_scale"]
    res, off = w.db()
    M = w.matrix()
    rec = workload_record(golden, "plain_scale", res, off, M, w)
    db = swmi.Database(res, off, 20)
    yield w, res, off, M, rec, db
    db.close()


@pytest.mark.parametrize("waves", [4, 8])
def test_plain_scale_full_size(swmi, orc, plain_db, waves):
    w, res, off, M, rec, db = plain_db
    qs = w.queries()
    db.set_opts(tier=1, strip=32, waves=waves)
    recomputed = 0
    for qi, q in enumerate(qs):
        e = query_record(rec, "plain_scale", qi, q)
        print(f"plain_scale full size: plan 1/32/{waves}, query {qi} ({len(q)} residues)", flush=True)
        ts, ti = db.topk(q, M, w.alpha, w.beta, 10)
        st = db.stats()
        assert st["tier"] == 1 and st["strip"] == 32 and st["waves"] == waves
        assert st["inter_cells"] > 0 and st["intra_pairs"] > 0
        got = db.search(q, M, w.alpha, w.beta)
        recomputed += db.stats()["recomputed_pairs"]
        check_full(orc, e, q, res, off, M, w, got, ts, ti,
                   f"plain_scale q{qi} waves {waves}", seed=2024 + qi)
    # the planted families reach past the fp16 ceiling: the exact int32
    # recompute ran and its results are part of the compared vectors
    assert recomputed > 0
    db.set_opts(reset=True)


def test_plain_scale_streamed_full_size(swmi, orc, plain_db, tmp_path):
    """plain_scale through an on-disk index (chunks of 128 M residues) with a
    1 GiB memory budget: the chunks stream through two device slots, all 20
    queries in one batch, every score vector against the oracle's digest."""
    w, res, off, M, rec, db = plain_db
    qs = w.queries()
    path = tmp_path / "plain_scale.swx"
    print("plain_scale streamed: writing the index", flush=True)
    swmi.sw_index_write(str(path), res, off, 20, 128 << 20)
    ix = swmi.Index(str(path), memory_budget=1 << 30)
    try:
        print("plain_scale streamed: search", flush=True)
        ts, ti, al = ix.search_batch(qs, M, w.alpha, w.beta, 10, all_scores=True)
        st = ix.stats()
    finally:
        ix.close()
    os.remove(path)
    assert st["resident"] == 0 and st["chunks"] >= 5 and st["bytes_loaded"] > (1 << 30)
    for qi, q in enumerate(qs):
        e = query_record(rec, "plain_scale", qi, q)
        check_full(orc, e, q, res, off, M, w, al[qi], ts[qi], ti[qi],
                   f"plain_scale streamed q{qi}", seed=3030 + qi)


def test_batched_full_size(swmi, orc, golden):
    w = sd.WORKLOADS["batched"]
    res, off = w.db()
    M = w.matrix()
    rec = workload_record(golden, "batched", res, off, M, w)
    qs = w.queries()
    assert len(qs) == 512
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
        keys = sorted(rec["queries"], key=int) or [str(x) for x in (3, 100, 511)]
        for key in keys:
            x = int(key)
            e = query_record(rec, "batched", x, qs[x])
            check_full(orc, e, qs[x], res, off, M, w, al[x], ts[x], ti[x], f"batched q{x}", seed=77 + x)
    finally:
        db.close()


def test_long_tail_full_size(swmi, orc, golden):
    """All 8 queries through the packed wave-per-pair kernel, fp16 plan, with
    each embedded homolog recomputed in int32."""
    w = sd.WORKLOADS["long_tail"]
    res, off = w.db()
    M = w.matrix()
    rec = workload_record(golden, "long_tail", res, off, M, w)
    qs = w.queries()
    db = swmi.Database(res, off, 20)
    try:
        for qi, q in enumerate(qs):
            e = query_record(rec, "long_tail", qi, q)
            print(f"long_tail full size: query {qi} ({len(q)} residues)", flush=True)
            ts, ti = db.topk(q, M, w.alpha, w.beta, 10)
            st = db.stats()
            assert st["intra_pairs"] == len(off) - 1 and st["inter_cells"] == 0
            # the embedded homolog scores above the fp16 ceiling
            assert st["recomputed_pairs"] >= (e["n_ge_1848"] if e else 1) >= 1
            got = db.search(q, M, w.alpha, w.beta)
            check_full(orc, e, q, res, off, M, w, got, ts, ti, f"long_tail q{qi}", seed=31 + qi)
    finally:
        db.close()


def test_served_full_size(swmi, orc, golden):
    """serving: 5,000,000 subjects (1.75 G residues) resident; requests of the
    serving query mix submitted together, so passes mix requests at
    different scan positions.  Each served top-10 equals the oracle's top-10
    over the whole database; a plain search of the same query gives the
    oracle's whole score vector."""
    w = sd.WORKLOADS["serving"]
    res, off = w.db()
    M = w.matrix()
    rec = workload_record(golden, "serving", res, off, M, w)
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
        assert sum(st["shared_passes"] for _, _, st in results) > 0, "no pass was shared"
        for x, (q, (ts, ti, st)) in enumerate(zip(qs, results)):
            e = query_record(rec, "serving", x, q)
            assert st["passes"] >= 1
            if e is not None:
                assert ts.tolist() == e["top_scores"] and ti.tolist() == e["top_idx"], \
                    f"served q{x}: top-{k} differs from the oracle's"
            else:
                exp = orc.search_subset(q, res, off, ti, M, w.alpha, w.beta)
                assert np.array_equal(ts, exp), f"served q{x}: top-k scores differ from the oracle"
            print(f"served full size: plain search of query {x}", flush=True)
            ps, pi = db.topk(q, M, w.alpha, w.beta, k)
            got = db.search(q, M, w.alpha, w.beta)
            check_full(orc, e, q, res, off, M, w, got, ps, pi, f"serving q{x} (plain)", seed=5 + x)
    finally:
        db.close()
