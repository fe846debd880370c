"""The entry point that allocates nothing (sw_db_search_dev_noalloc), called
through the C ABI and checked bit for bit against sw_db_search_dev on the same
inputs: two calls in a row, the second with a smaller query, so the second
runs on scratch contents the first left behind.

The database mixes lane-per-subject groups, a long list (a fixed cut at 1,500
residues) and a planted homolog of the first query, whose score passes the
fp16 tier's ceiling: the overflow list and the int32 recompute run inside the
fixed scratch too.
"""
import numpy as np
import pytest

import synthdata as sd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1404_4152_amd as swmi
    swmi.lib()
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    rng = np.random.Generator(np.random.PCG64(4242))
    q1 = sd.random_residues(rng, 600)
    q2 = sd.random_residues(rng, 150)
    res, off = sd.make_db(20000, 350, 20, 5000, seed=91)
    # a 90%-identity copy of q1 replaces subject 7: its score passes 1,848
    res, off = sd.rebuild_db(res, off, {7: sd.mutate(rng, q1, 0.9)})
    db = swmi.Database(res, off, 20, long_threshold=1500, device=0)
    yield torch, swmi, db, res, off, (q1, q2)
    db.close()


def run_pair(torch, swmi, db, q, M, alpha, beta, stream_ptr):
    n = swmi.sw_db_size(db.h)
    qd = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    ref = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    got = torch.full((n,), -9, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()   # the library's own stream (stream_ptr None) does not wait for torch's
    swmi.sw_db_search_dev(db.h, q, M, alpha, beta, ref.data_ptr(), stream=stream_ptr)
    st_ref = db.stats()
    swmi.sw_db_search_dev_noalloc(db.h, qd.data_ptr(), len(q), M, alpha, beta, got.data_ptr(),
                                  stream=stream_ptr)
    st = db.stats()
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy(), st_ref, st


@pytest.mark.parametrize("use_torch_stream", [True, False])
def test_noalloc_equals_search_dev_twice(env, use_torch_stream):
    torch, swmi, db, res, off, (q1, q2) = env
    M = sd.blosum_style_matrix()
    sptr = torch.cuda.current_stream().cuda_stream if use_torch_stream else None
    for q in (q1, q2):   # the second call has the smaller input
        print(f"no-alloc search: query of {len(q)} residues, torch stream {use_torch_stream}",
              flush=True)
        ref, got, st_ref, st = run_pair(torch, swmi, db, q, M, 2, 12, sptr)
        bad = np.flatnonzero(ref != got)
        assert bad.size == 0, (f"{bad.size} scores differ, first ids {bad[:5].tolist()}: "
                               f"{got[bad[:5]].tolist()} vs {ref[bad[:5]].tolist()}")
        assert (ref >= 0).all()
        assert st["tier"] == st_ref["tier"] and st["inter_cells"] > 0 and st["intra_pairs"] > 0
        if q is q1:
            assert st_ref["recomputed_pairs"] >= 1 and ref[7] >= 1848


def test_noalloc_high_alpha_and_int16(env):
    """alpha above the fp16 tier's range: the int16 plan, same scratch."""
    torch, swmi, db, res, off, (q1, q2) = env
    M = sd.blosum_style_matrix()
    ref, got, st_ref, st = run_pair(torch, swmi, db, q2, M, 40, 60, None)
    assert st["tier"] == 2
    assert np.array_equal(ref, got)


def test_noalloc_rejects_oversize_before_gpu_work(env):
    """A query whose profile alone exceeds the fixed scratch fails with
    SW_EINVAL on the host; nothing is launched (the query buffer is never read)."""
    torch, swmi, db, res, off, (q1, q2) = env
    M = sd.blosum_style_matrix()
    qd = torch.zeros(16, dtype=torch.uint8, device="cuda")
    out = torch.zeros(swmi.sw_db_size(db.h), dtype=torch.int32, device="cuda")
    with pytest.raises(swmi.SwError) as ei:
        swmi.sw_db_search_dev_noalloc(db.h, qd.data_ptr(), 1 << 24, M, 2, 12, out.data_ptr())
    assert ei.value.code == -1 and "no-allocation scratch" in str(ei.value)
