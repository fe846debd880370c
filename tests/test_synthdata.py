"""The seeded generators are deterministic and have the stated shapes."""
import numpy as np

import synthdata as sd


def test_matrix_is_symmetric_and_blosum_like():
    M = sd.blosum_style_matrix()
    assert M.dtype == np.int8 and M.shape == (20, 20)
    assert (M == M.T).all()
    assert M.min() >= -4 and M.max() <= 11
    assert (np.diag(M) > 0).all()
    f = sd.background_frequencies()
    assert float((f[:, None] * f[None, :] * M).sum()) < 0   # random pairs score negative
    assert sd.sha256(M) == sd.sha256(sd.blosum_style_matrix())


def test_db_determinism_and_shape():
    r1, o1 = sd.make_db(2000, 350, 20, 2000)
    r2, o2 = sd.make_db(2000, 350, 20, 2000)
    assert sd.sha256(r1, o1) == sd.sha256(r2, o2)
    lens = np.diff(o1)
    assert lens.min() >= 20 and lens.max() <= 2000
    assert 300 < lens.mean() < 400
    assert r1.max() < 20
    freq = np.bincount(r1, minlength=20) / len(r1)
    assert np.abs(freq - sd.background_frequencies()).max() < 0.005


def test_sorted_db_is_sorted():
    _, o = sd.make_db(5000, 350, 20, 35000, sort=True)
    assert (np.diff(np.diff(o)) >= 0).all()


def test_queries_and_homologs():
    qs = sd.make_queries([144, 189])
    assert [len(q) for q in qs] == [144, 189]
    r, o = sd.make_db(50, 350, 20, 2000)
    r2, o2 = sd.plant_homologs(r, o, qs, [3, 7])
    assert len(o2) == 51
    h = r2[o2[3]:o2[4]]
    assert 120 < len(h) < 170
    assert sd.sha256(r2[o2[0]:o2[3]]) == sd.sha256(r[o[0]:o[3]])


def test_workload_table():
    w = sd.WORKLOADS["plain_scale"]
    assert w.query_lengths == sd.SCALE_QUERY_LENGTHS and sum(w.query_lengths) == 41752
    assert len(sd.WORKLOADS["batched"].query_lengths) == 512
    assert sd.WORKLOADS["long_tail"].query_lengths == [1000, 1571, 2143, 2714, 3286, 3857, 4429, 5000]
