"""The on-disk index (sw_index_write) needs no GPU: written here and read
back with numpy, independently of the library.  Checked: the header, that
the chunks partition the database, that they follow the length order and
respect the chunk size, that each chunk lists its subjects in ascending
database order with their residues intact, and the packed group tables
(every short subject in exactly one group slot, padding to whole chunks of
rows, pair codes lo * R + hi with the zero-score pad code R - 1)."""
import os

import numpy as np
import pytest

import synthdata as sd

HDR = np.dtype([("magic", "S8"), ("version", "<i4"), ("alphabet", "<i4"), ("n_seqs", "<i8"),
                ("total_res", "<i8"), ("n_chunks", "<i8"), ("chunk_residues", "<i8"),
                ("reserved", "<i8", 4)])
ENTRY = np.dtype([("file_off", "<i8"), ("bytes", "<i8"), ("n_seqs", "<i8"), ("total_res", "<i8"),
                  ("device_bytes", "<i8")])
HEAD = np.dtype([("n_seqs", "<i8"), ("total_res", "<i8"), ("max_len", "<i8"), ("long_res", "<i8"),
                 ("long_threshold", "<i8"), ("inter_res", "<i8"), ("inter_padded_rows", "<i8"),
                 ("n_codes", "<i8"), ("n_groups", "<i4"), ("max_rows", "<i4"), ("n_long", "<i4"),
                 ("fixed_cut", "<i4")])


def al64(x):
    return (x + 63) // 64 * 64


def read_chunk(buf, off):
    h = np.frombuffer(buf, HEAD, 1, off)[0]
    n, tot, ng, nl, nc = int(h["n_seqs"]), int(h["total_res"]), int(h["n_groups"]), int(h["n_long"]), int(h["n_codes"])
    o = al64(HEAD.itemsize)
    out = {"head": h}
    for name, dt, cnt in [("ids", "<i4", n), ("offsets", "<i8", n + 1), ("residues", "u1", tot),
                          ("long_ids", "<i4", nl), ("grp_rows", "<i4", ng), ("grp_ids", "<i4", ng * 128),
                          ("grp_res_prefix", "<i8", ng + 1), ("gbase", "<i8", ng), ("codes", "<u2", nc)]:
        out[name] = np.frombuffer(buf, dt, cnt, off + o)
        o = al64(o + cnt * np.dtype(dt).itemsize)
    out["end"] = o
    return out


@pytest.fixture(scope="module")
def swmi():
    import paper_1404_4152_amd as p
    if not os.path.exists(p.LIB_PATH):
        pytest.skip("libswmi.so not built")
    p.lib()
    return p


@pytest.mark.parametrize("n,chunk", [(3000, 40_000), (200_000, 30_000_000), (200_000, 12_000_000),
                                     (1, 10), (50, 1)])
def test_index_file_layout(swmi, tmp_path, n, chunk):
    res, off = sd.make_db(n, 300, 0, 9000, seed=n)   # zero-length subjects included
    lens = np.diff(off)
    path = tmp_path / "db.swx"
    swmi.sw_index_write(str(path), res, off, 20, chunk)
    buf = path.read_bytes()
    h = np.frombuffer(buf, HDR, 1, 0)[0]
    assert h["magic"] == b"SWMIIDX1" and h["version"] == 1 and h["alphabet"] == 20
    assert h["n_seqs"] == n and h["total_res"] == off[-1] and h["chunk_residues"] == chunk
    nchunks = int(h["n_chunks"])
    layout = int(h["reserved"][0])
    table = np.frombuffer(buf, ENTRY, nchunks, HDR.itemsize)
    seen = []
    prev_max = -1
    # the length order (stable), dealt round-robin over the chunks (layout 1)
    # or cut into consecutive runs (layout 0)
    rank_order = np.argsort(lens, kind="stable")
    if layout == 1:
        assert off[-1] > chunk and 4 * lens.max() <= chunk and nchunks >= 2
    else:
        assert layout == 0
    R = 21
    for e in table:
        c = read_chunk(buf, int(e["file_off"]))
        assert c["end"] == e["bytes"] and int(e["file_off"]) % 64 == 0
        ids = c["ids"].astype(np.int64)
        assert (np.diff(ids) > 0).all()                         # ascending database order
        clen = lens[ids]
        assert np.array_equal(np.diff(c["offsets"]), clen)
        assert clen.sum() <= chunk or len(ids) == 1
        if layout == 1:
            assert np.array_equal(ids, np.sort(rank_order[len(seen)::nchunks]))
        else:
            assert clen.min() >= prev_max                       # length order across chunks
            prev_max = clen.max()
        for i in np.random.default_rng(0).choice(len(ids), size=min(50, len(ids)), replace=False):
            a, b = c["offsets"][i], c["offsets"][i + 1]
            assert np.array_equal(c["residues"][a:b], res[off[ids[i]]:off[ids[i] + 1]])
        # packed tables: local ids of the groups and the long list cover the chunk once
        slots = c["grp_ids"][c["grp_ids"] >= 0]
        both = np.concatenate([slots, c["long_ids"]])
        assert np.array_equal(np.sort(both), np.arange(len(ids)))
        ng = int(c["head"]["n_groups"])
        for g in range(min(ng, 3)):
            rows = int(c["grp_rows"][g])
            assert rows % 4 == 0
            members = c["grp_ids"][g * 128:(g + 1) * 128]
            assert rows >= max(int(clen[m]) for m in members if m >= 0)
            codes = c["codes"][int(c["gbase"][g]):int(c["gbase"][g]) + rows * 64]
            lane = 5
            lo, hi = members[lane], members[64 + lane]
            for i in range(rows):
                v = int(codes[(i // 4) * 256 + lane * 4 + i % 4])
                a = int(c["residues"][c["offsets"][lo] + i]) if lo >= 0 and i < clen[lo] else R - 1
                b = int(c["residues"][c["offsets"][hi] + i]) if hi >= 0 and i < clen[hi] else R - 1
                assert v == a * R + b
        seen.append(ids)
    allids = np.concatenate(seen) if seen else np.zeros(0, np.int64)
    assert np.array_equal(np.sort(allids), np.arange(n))


def test_index_write_rejects_bad_input(swmi, tmp_path):
    res, off = sd.make_db(10, 50, 1, 100, seed=3)
    with pytest.raises(swmi.SwError):
        swmi.sw_index_write(str(tmp_path / "a"), res, off, 20, 0)
    bad = res.copy()
    bad[3] = 25
    with pytest.raises(swmi.SwError):
        swmi.sw_index_write(str(tmp_path / "b"), bad, off, 20, 1000)
    with pytest.raises(swmi.SwError):
        swmi.sw_index_write(str(tmp_path / "no" / "such" / "dir"), res, off, 20, 1000)
