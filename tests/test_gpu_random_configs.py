"""Seeded random configurations through every route, against the oracle.

Each case draws a database (size, length range, alphabet, zero-length
subjects), a matrix, gap penalties, a saturation threshold and a plan knob,
then compares sw_db_search, sw_db_topk and sw_db_search_batch with the
oracle element by element.  The draws cover what the fixed cases cover one
at a time, in combination: databases small enough to be all long list
(packed or int32 by columns per lane) or large enough for lane-per-subject
groups, thresholds low enough that both narrow kernels flag (and the packed
one recomputes in its own launch), alpha past the fp16 frame's range (the
planner's int16 tier), queries of one to several passes.  The draws are
fixed by the seeds, so a failure names a reproducible case.
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


def draw_case(seed):
    rng = np.random.Generator(np.random.PCG64(90_000 + seed))
    A = int(rng.choice([3, 20, 20, 24]))
    n = int(rng.choice([1, 40, 700, 3000, 9000]))
    hi = int(rng.choice([30, 300, 1500]))
    lens = rng.integers(0, hi + 1, size=n)
    if n > 5 and rng.random() < 0.5:
        lens[rng.integers(0, n, size=max(1, n // 50))] = 0
    res, off = sd.pack_sequences([sd.uniform_residues(rng, int(L), A) for L in lens])
    M = sd.blosum_style_matrix() if A == 20 and rng.random() < 0.5 else sd.random_matrix(rng, A)
    alpha = int(rng.choice([0, 1, 2, 3, 28, 29, 40]))
    beta = alpha + int(rng.choice([0, 1, 10, 25]))
    thr = int(rng.choice([0, 0, 15, 60]))
    route = int(rng.choice([0, 0, -1, 1]))
    tier = int(rng.choice([0, 0, 1, 2]))
    qlens = [int(x) for x in rng.integers(1, 1300, size=3)]
    qs = [sd.uniform_residues(rng, L, A) for L in qlens]
    k = int(rng.choice([1, 10, 37]))
    return dict(A=A, n=n, res=res, off=off, M=M, alpha=alpha, beta=beta, thr=thr, route=route,
                tier=tier, qs=qs, k=k)


@pytest.mark.parametrize("seed", range(64))
def test_random_config(swmi, orc, seed):
    c = draw_case(seed)
    what = (f"seed {seed}: A {c['A']} n {c['n']} alpha {c['alpha']} beta {c['beta']} thr {c['thr']} "
            f"route {c['route']} tier {c['tier']} qlens {[len(q) for q in c['qs']]} k {c['k']}")
    print(what, flush=True)
    res, off, M = c["res"], c["off"], c["M"]
    db = swmi.Database(res, off, c["A"], long_threshold=c["route"])
    try:
        db.set_opts(tier=c["tier"], sat_threshold=c["thr"])
        exps = [orc.search(q, res, off, M, c["alpha"], c["beta"]) for q in c["qs"]]
        for q, exp in zip(c["qs"], exps):
            got = db.search(q, M, c["alpha"], c["beta"])
            bad = np.flatnonzero(got != exp)
            assert bad.size == 0, (what, len(q), bad[:5].tolist(), got[bad[:5]].tolist(), exp[bad[:5]].tolist())
            ts, ti = db.topk(q, M, c["alpha"], c["beta"], c["k"])
            es, ei = oracle.topk(exp, c["k"])
            assert np.array_equal(ts, es) and np.array_equal(ti, ei), (what, "topk", len(q))
        ts, ti, al = db.search_batch(c["qs"], M, c["alpha"], c["beta"], c["k"], all_scores=True)
        for x, exp in enumerate(exps):
            assert np.array_equal(al[x], exp), (what, "batch", x)
            es, ei = oracle.topk(exp, c["k"])
            assert np.array_equal(ts[x], es) and np.array_equal(ti[x], ei), (what, "batch topk", x)
    finally:
        db.close()
