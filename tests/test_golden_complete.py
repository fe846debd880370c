"""The stored oracle results at full size (tests/golden/full_size.json) are
complete and were written for exactly the inputs synthdata draws today: every
query of plain_scale and long_tail, the seeded sample of batched, and the
served test's queries, each with a score-vector digest and a top-10 whose
order is (score descending, index ascending).  No GPU needed."""
import json
import os
import sys

import numpy as np
import pytest

import synthdata as sd

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_full_size as mfs  # noqa: E402

with open(os.path.join(HERE, "golden", "full_size.json")) as f:
    DOC = json.load(f)


@pytest.mark.parametrize("name", ["long_tail", "batched", "serving", "plain_scale"])
def test_full_size_records_complete(name):
    rec = DOC.get(name)
    assert rec is not None, f"no {name} records"
    w = sd.WORKLOADS[name]
    res, off = w.db()
    assert rec["db_sha256"] == sd.sha256(res, off)
    assert rec["matrix_sha256"] == sd.sha256(w.matrix())
    assert (rec["alpha"], rec["beta"], rec["n_subjects"], rec["residues"]) == \
        (w.alpha, w.beta, len(off) - 1, int(off[-1]))
    idx, qs = mfs.workload_queries(name)
    missing = [i for i in idx if str(i) not in rec["queries"]]
    assert not missing, f"{name}: no oracle record for queries {missing}"
    for i, q in zip(idx, qs):
        e = rec["queries"][str(i)]
        assert e["query_sha256"] == sd.sha256(q) and e["qlen"] == len(q)
        assert len(e["scores_sha256"]) == 64
        ts, ti = np.array(e["top_scores"]), np.array(e["top_idx"])
        assert len(ts) == rec["k"] == len(ti)
        # (score desc, index asc), the top-10 no higher than the record's max
        assert ts[0] == e["max"]
        assert all((ts[j] > ts[j + 1]) or (ts[j] == ts[j + 1] and ti[j] < ti[j + 1])
                   for j in range(len(ts) - 1))
