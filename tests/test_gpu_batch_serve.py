"""GPU tests of the batched (graph-captured) path, the autotuner and the server.

Every result is compared exactly with the CPU oracle; the server's results
must be identical whether a request runs alone or mixed with others.
"""
import json
import os
import threading
import time

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


def random_db(rng, n, A, lo, hi):
    lens = rng.integers(lo, hi + 1, size=n)
    lens[::97] = 0
    return sd.pack_sequences([rng.integers(0, A, size=int(L)).astype(np.uint8) for L in lens])


def oracle_topk(orc, q, res, off, M, a, b, k):
    return oracle.topk(orc.search(q, res, off, M, a, b), k)


def test_batch_graph_replays_match_oracle(swmi, orc):
    """Replays of one captured batch shape, with different queries each time and
    eager work in between, all match the oracle and the eager launch."""
    rng = np.random.Generator(np.random.PCG64(41))
    M = sd.blosum_style_matrix()
    res, off = random_db(rng, 3000, 20, 1, 400)
    db = swmi.Database(res, off, 20, long_threshold=300)
    try:
        for rep in range(4):
            qs = [sd.random_residues(rng, int(L)) for L in rng.integers(20, 700, size=6)]
            print(f"graph replay {rep}", flush=True)
            ts, ti, al = db.search_batch(qs, M, 2, 12, 10, all_scores=True)
            st = db.stats()
            assert st["graphed"] == 1
            for x, q in enumerate(qs):
                exp = orc.search(q, res, off, M, 2, 12)
                assert np.array_equal(al[x], exp), f"replay {rep} query {x}"
                es, ei = oracle.topk(exp, 10)
                assert np.array_equal(ts[x], es) and np.array_equal(ti[x], ei)
            # eager work between replays
            q0 = sd.random_residues(rng, 90)
            assert np.array_equal(db.search(q0, M, 2, 12), orc.search(q0, res, off, M, 2, 12))
        db.set_opts(graph=-1)
        ts2, ti2, al2 = db.search_batch(qs, M, 2, 12, 10, all_scores=True)
        assert db.stats()["graphed"] == 0
        assert np.array_equal(al2, al) and np.array_equal(ts2, ts) and np.array_equal(ti2, ti)
    finally:
        db.close()


def test_autotune_and_cache(swmi, orc, tmp_path):
    rng = np.random.Generator(np.random.PCG64(43))
    M = sd.blosum_style_matrix()
    res, off = random_db(rng, 6000, 20, 1, 300)
    path = str(tmp_path / "tune.json")
    db = swmi.Database(res, off, 20, long_threshold=-1)
    try:
        swmi.sw_db_autotune(db.h, M, 2, 12, [100, 600], path)
        text = json.load(open(path))
        # buckets of 100 and 600 residues, and the batch entry (bucket -1)
        assert sorted(e["bucket"] for e in text["entries"]) == [-1, 1, 4]
        for e in text["entries"]:
            assert e["tier"] in (1, 2) and e["strip"] in (16, 32, 64) and e["gcups"] > 0
        q = sd.random_residues(rng, 600)
        assert np.array_equal(db.search(q, M, 2, 12), orc.search(q, res, off, M, 2, 12))
        # a launch of several queries runs the batch entry's plan
        batch = next(e for e in text["entries"] if e["bucket"] == -1)
        qs = [sd.random_residues(rng, L) for L in (100, 600, 333)]
        ts, ti, al = db.search_batch(qs, M, 2, 12, 5, all_scores=True)
        st = db.stats()
        assert (st["tier"], st["strip"], st["waves"]) == (batch["tier"], batch["strip"], batch["waves"])
        for x, qx in enumerate(qs):
            assert np.array_equal(al[x], orc.search(qx, res, off, M, 2, 12))
    finally:
        db.close()
    db = swmi.Database(res, off, 20, long_threshold=-1)
    try:
        mtime = os.path.getmtime(path)
        swmi.sw_db_autotune(db.h, M, 2, 12, [100, 600], path)   # read from the cache
        assert os.path.getmtime(path) == mtime
        q = sd.random_residues(rng, 120)
        assert np.array_equal(db.search(q, M, 2, 12), orc.search(q, res, off, M, 2, 12))
    finally:
        db.close()


def serve_db(swmi, rng):
    res, off = random_db(rng, 4000, 20, 1, 500)
    # subjects over 380 residues form the long list: one more scan position
    return res, off, swmi.Database(res, off, 20, long_threshold=380)


def test_server_alone_equals_mixed_equals_oracle(swmi, orc):
    rng = np.random.Generator(np.random.PCG64(47))
    M = sd.blosum_style_matrix()
    res, off, db = serve_db(swmi, rng)
    qs = [sd.random_residues(rng, int(L)) for L in rng.integers(30, 900, size=10)]
    k = 12
    try:
        srv = swmi.sw_server_start(db.h, chunk_groups=4, max_active=6)
        try:
            alone = []
            for q in qs:
                t = swmi.sw_server_submit(srv, q, M, 2, 12, k)
                ts, ti, st = swmi.sw_server_wait(srv, t, k)
                assert st["passes"] >= 1
                alone.append((ts, ti))
            # mixed: submitted from several threads, staggered, more than max_active
            tickets = [None] * len(qs)

            def submit(x):
                time.sleep(0.002 * x)
                tickets[x] = swmi.sw_server_submit(srv, qs[x], M, 2, 12, k)

            th = [threading.Thread(target=submit, args=(x,)) for x in range(len(qs))]
            for t in th:
                t.start()
            for t in th:
                t.join()
            mixed = [swmi.sw_server_wait(srv, t, k)[:2] for t in tickets]
        finally:
            swmi.sw_server_stop(srv)
        for x, q in enumerate(qs):
            es, ei = oracle_topk(orc, q, res, off, M, 2, 12, k)
            assert np.array_equal(alone[x][0], es) and np.array_equal(alone[x][1], ei), f"alone {x}"
            assert np.array_equal(mixed[x][0], alone[x][0]) and np.array_equal(mixed[x][1], alone[x][1])
        # the database serves plain searches again once the server is gone
        q = qs[0]
        assert np.array_equal(db.search(q, M, 2, 12), orc.search(q, res, off, M, 2, 12))
    finally:
        db.close()


def test_server_tiny_budget_queues_but_completes(swmi, orc):
    rng = np.random.Generator(np.random.PCG64(53))
    M = sd.blosum_style_matrix()
    res, off, db = serve_db(swmi, rng)
    qs = [sd.random_residues(rng, int(L)) for L in rng.integers(30, 300, size=6)]
    # charged per request: its profile (21 rows x qlen rounded up to 32) and top-k
    per_request = 21 * 320 + 5 * 12
    try:
        srv = swmi.sw_server_start(db.h, memory_budget=per_request + 100, chunk_groups=8)
        try:
            tickets = [swmi.sw_server_submit(srv, q, M, 2, 12, 5) for q in qs]
            out = [swmi.sw_server_wait(srv, t, 5) for t in tickets]
        finally:
            swmi.sw_server_stop(srv)
        for q, (ts, ti, st) in zip(qs, out):
            es, ei = oracle_topk(orc, q, res, off, M, 2, 12, 5)
            assert np.array_equal(ts, es) and np.array_equal(ti, ei)
        assert max(st["queue_ms"] for _, _, st in out) > 0
    finally:
        db.close()


def test_server_mixed_schemes_share_passes(swmi, orc):
    """Requests with different gap penalties and matrices share passes:
    alpha up to 28 runs in the fp16 tier, larger alpha (up to past the fp16
    frame's limit of 53) in the int16 sub-pass of the same passes.  A burst
    spanning many passes (small chunks) must give every request the same
    top-k as running alone, and as the oracle, and requests must have shared
    passes with others."""
    rng = np.random.Generator(np.random.PCG64(71))
    M = sd.blosum_style_matrix()
    M2 = sd.random_matrix(rng, 20, lo=-5, hi=8, symmetric=False)
    res, off, db = serve_db(swmi, rng)
    schemes = [(M, 2, 12), (M2, 1, 11), (M, 28, 40), (M2, 29, 29), (M, 40, 60), (M, 60, 80),
               (M2, 0, 0), (M, 3, 9)]
    qs = [sd.random_residues(rng, int(L)) for L in rng.integers(40, 900, size=len(schemes))]
    ks = [5, 12, 7, 3, 10, 4, 9, 6]
    try:
        srv = swmi.sw_server_start(db.h, chunk_groups=2, max_active=16)
        try:
            alone = []
            for q, (m, a, b), k in zip(qs, schemes, ks):
                t = swmi.sw_server_submit(srv, q, m, a, b, k)
                alone.append(swmi.sw_server_wait(srv, t, k))
            # the burst: half now, half once the first ones are under way
            tickets = [swmi.sw_server_submit(srv, q, m, a, b, k)
                       for q, (m, a, b), k in list(zip(qs, schemes, ks))[:4]]
            time.sleep(0.003)
            tickets += [swmi.sw_server_submit(srv, q, m, a, b, k)
                        for q, (m, a, b), k in list(zip(qs, schemes, ks))[4:]]
            mixed = [swmi.sw_server_wait(srv, t, k) for t, k in zip(tickets, ks)]
        finally:
            swmi.sw_server_stop(srv)
        shared = [st["shared_passes"] for _, _, st in mixed]
        print("passes", [st["passes"] for _, _, st in mixed], "shared", shared, flush=True)
        assert sum(1 for x in shared if x > 0) >= len(qs) - 1, shared
        for x, (q, (m, a, b), k) in enumerate(zip(qs, schemes, ks)):
            es, ei = oracle_topk(orc, q, res, off, m, a, b, k)
            assert np.array_equal(alone[x][0], es) and np.array_equal(alone[x][1], ei), \
                f"alone {x} alpha {a}"
            assert np.array_equal(mixed[x][0], es) and np.array_equal(mixed[x][1], ei), \
                f"mixed {x} alpha {a}"
    finally:
        db.close()


def test_server_budget_lets_small_requests_pass(swmi, orc):
    """A long query that does not fit the memory budget beside another waits,
    while a short one submitted after it is admitted at once."""
    rng = np.random.Generator(np.random.PCG64(73))
    M = sd.blosum_style_matrix()
    res, off, db = serve_db(swmi, rng)
    qa, qb, qc = (sd.random_residues(rng, L) for L in (2000, 2000, 50))
    k = 4
    long_bytes = 21 * 2016 + 12 * k
    short_bytes = 21 * 64 + 12 * k
    try:
        srv = swmi.sw_server_start(db.h, memory_budget=long_bytes + short_bytes + 100,
                                   chunk_groups=1, max_active=8)
        try:
            ta, tb, tc = (swmi.sw_server_submit(srv, q, M, 2, 12, k) for q in (qa, qb, qc))
            ra, rb, rc = (swmi.sw_server_wait(srv, t, k) for t in (ta, tb, tc))
        finally:
            swmi.sw_server_stop(srv)
        sa, sb, sc_ = ra[2], rb[2], rc[2]
        print("queue ms", sa["queue_ms"], sb["queue_ms"], sc_["queue_ms"], "A total",
              sa["total_ms"], flush=True)
        assert sc_["queue_ms"] < sb["queue_ms"]
        assert sb["queue_ms"] >= sa["total_ms"] - 5.0   # B waited for A to complete
        for q, (ts, ti, _) in zip((qa, qb, qc), (ra, rb, rc)):
            es, ei = oracle_topk(orc, q, res, off, M, 2, 12, k)
            assert np.array_equal(ts, es) and np.array_equal(ti, ei)
    finally:
        db.close()


def test_server_backpressure_and_errors(swmi):
    rng = np.random.Generator(np.random.PCG64(59))
    M = sd.blosum_style_matrix()
    res, off, db = serve_db(swmi, rng)
    try:
        srv = swmi.sw_server_start(db.h, max_active=1, queue_capacity=1, chunk_groups=2)
        busy = 0
        accepted = []
        try:
            for _ in range(30):
                try:
                    accepted.append(swmi.sw_server_submit(srv, sd.random_residues(rng, 800), M, 2, 12, 3))
                except swmi.SwError as e:
                    assert e.code == swmi.SW_EBUSY
                    busy += 1
            with pytest.raises(swmi.SwError) as e:
                swmi.sw_server_wait(srv, 987654321, 3)
            assert e.value.code == swmi.SW_ENOTFOUND
            with pytest.raises(swmi.SwError) as e:
                swmi.sw_server_submit(srv, np.array([30], np.uint8), M, 2, 12, 3)
            assert e.value.code == swmi.SW_EINVAL
            for t in accepted:
                swmi.sw_server_wait(srv, t, 3)
        finally:
            swmi.sw_server_stop(srv)
        assert busy > 0 and len(accepted) >= 1
        # a plain search while a server runs is refused; after stop it works
        srv = swmi.sw_server_start(db.h)
        try:
            with pytest.raises(swmi.SwError) as e:
                db.search(np.array([1, 2], np.uint8), M, 2, 12)
            assert e.value.code == swmi.SW_EBUSY
        finally:
            swmi.sw_server_stop(srv)
        db.search(np.array([1, 2], np.uint8), M, 2, 12)
    finally:
        db.close()


def test_server_stop_with_pending_requests(swmi):
    rng = np.random.Generator(np.random.PCG64(61))
    M = sd.blosum_style_matrix()
    res, off, db = serve_db(swmi, rng)
    try:
        srv = swmi.sw_server_start(db.h, max_active=1, chunk_groups=1)
        tickets = [swmi.sw_server_submit(srv, sd.random_residues(rng, 1500), M, 2, 12, 3)
                   for _ in range(8)]
        codes = []

        def waiter(t):
            try:
                swmi.sw_server_wait(srv, t, 3)
                codes.append(0)
            except swmi.SwError as e:
                codes.append(e.code)

        th = [threading.Thread(target=waiter, args=(t,)) for t in tickets]
        for t in th:
            t.start()
        time.sleep(0.05)
        swmi.sw_server_stop(srv)
        for t in th:
            t.join()
        assert len(codes) == 8
        assert set(codes) <= {0, swmi.SW_ESTOPPED} and swmi.SW_ESTOPPED in codes
    finally:
        db.close()


def test_injected_allocation_failure(swmi):
    rng = np.random.Generator(np.random.PCG64(67))
    res, off = random_db(rng, 100, 20, 1, 50)
    os.environ["SWMI_FAIL_ALLOC"] = "1"
    try:
        with pytest.raises(swmi.SwError) as e:
            swmi.Database(res, off, 20)
        assert e.value.code == swmi.SW_ENOMEM
    finally:
        del os.environ["SWMI_FAIL_ALLOC"]
    db = swmi.Database(res, off, 20)
    db.close()
