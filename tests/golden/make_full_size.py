"""Write tests/golden/full_size.json: the oracle's full score vectors at the
benchmark's full sizes, stored as SHA-256 digests plus the oracle's top-10.

Only the CPU oracle (``oracle/``) computes anything here; ``synthdata/``
draws the inputs.  Nothing comes from the GPU library.

Per query the record holds:
  - ``scores_sha256``: SHA-256 of the full int32 score vector (little-endian,
    database order) that ``oracle.search`` returns (Eq. 1 of section II.A);
  - ``top_scores`` / ``top_idx``: ``oracle.topk`` of that vector (score
    descending, then ascending database index);
  - ``max``, ``n_ge_1848``: the largest score and how many subjects reach
    1,848 (the fp16 tier's threshold at alpha = 2), for the reader.

Workloads and queries:
  - plain_scale: all 20 queries x 2,000,000 subjects;
  - long_tail:   all 8 queries x 20,000 subjects;
  - batched:     a seeded sample of 16 of the 512 queries x 500,000 subjects;
  - serving:     the 6 queries of the served full-size test x 5,000,000.

The run takes hours of CPU.  It is resumable: records whose input digests
match are kept, so an interrupted run continues where it stopped.

    python tests/golden/make_full_size.py [--threads N] [--only NAME ...]
        [--queries I ...] [--out PATH] [--slices N]

--queries limits the run to those query indices; --out writes the records to
another file (for example on a machine with more cores), whose records
--merge PATH later copies into this one.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle            # noqa: E402
import synthdata as sd   # noqa: E402

OUT = os.path.join(HERE, "full_size.json")
K = 10
# Seeded sample of the batched workload's 512 queries.
BATCHED_SAMPLE_SEED = 4096
BATCHED_SAMPLE = 16
SERVED_QUERIES = 6
ORDER = ("long_tail", "batched", "serving", "plain_scale")


def batched_sample() -> list[int]:
    rng = np.random.Generator(np.random.PCG64(BATCHED_SAMPLE_SEED))
    return sorted(int(x) for x in rng.choice(512, size=BATCHED_SAMPLE, replace=False))


def workload_queries(name: str):
    """(query indices, query arrays) checked for one workload."""
    if name == "serving":
        qs = sd.serving_queries(SERVED_QUERIES)
        return list(range(len(qs))), qs
    qs = sd.WORKLOADS[name].queries()
    if name == "batched":
        idx = batched_sample()
        return idx, [qs[i] for i in idx]
    return list(range(len(qs))), qs


def vector_sha256(scores: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(scores, dtype="<i4").tobytes()).hexdigest()


def load(path: str = OUT) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save(doc: dict, path: str = OUT) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, path)


def merge(src: str) -> None:
    """Copy the query records of another run's file into OUT, for workloads
    whose input digests agree."""
    doc, other = load(), load(src)
    for name, rec in other.items():
        if name == "about":
            continue
        mine = doc.setdefault(name, {})
        keys = ("db_sha256", "matrix_sha256", "alpha", "beta", "n_subjects", "residues", "k")
        if mine and any(mine.get(x) != rec.get(x) for x in keys):
            raise SystemExit(f"{name}: inputs of {src} differ from {OUT}'s")
        for x in keys:
            mine[x] = rec[x]
        mine.setdefault("queries", {}).update(rec.get("queries", {}))
        print(f"[golden] merged {len(rec.get('queries', {}))} {name} records", flush=True)
    save(doc)


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--only", nargs="*", default=None)
    ap.add_argument("--queries", nargs="*", type=int, default=None)
    ap.add_argument("--out", default=OUT)
    ap.add_argument("--merge", default=None)
    ap.add_argument("--slices", type=int, default=1,
                    help="compute each vector in this many slices of the database, printing each")
    args = ap.parse_args()
    if args.merge:
        merge(args.merge)
        return
    orc = oracle.load()
    doc = load(args.out)
    doc["about"] = ("Oracle score-vector digests and top-10 at full size; written by "
                    "tests/golden/make_full_size.py, which calls only oracle/.")
    for name in ORDER:
        if args.only and name not in args.only:
            continue
        w = sd.WORKLOADS[name]
        t0 = time.time()
        res, off = w.db()
        M = w.matrix()
        db_sha = sd.sha256(res, off)
        rec = doc.setdefault(name, {})
        if rec.get("db_sha256") != db_sha or rec.get("matrix_sha256") != sd.sha256(M):
            rec.clear()
        rec.update({"db_sha256": db_sha, "matrix_sha256": sd.sha256(M),
                    "alpha": w.alpha, "beta": w.beta, "n_subjects": len(off) - 1,
                    "residues": int(off[-1]), "k": K})
        entries = rec.setdefault("queries", {})
        idx, qs = workload_queries(name)
        print(f"[golden] {name}: {len(qs)} queries, {len(off) - 1} subjects "
              f"(inputs in {time.time() - t0:.1f}s)", flush=True)
        for i, q in zip(idx, qs):
            if args.queries is not None and i not in args.queries:
                continue
            key = str(i)
            q_sha = sd.sha256(q)
            if entries.get(key, {}).get("query_sha256") == q_sha:
                continue
            t1 = time.time()
            if args.slices > 1:
                # the same per-subject scores, computed in slices of the
                # database so that progress shows while a long query runs
                n = len(off) - 1
                parts = []
                for x in range(args.slices):
                    lo, hi = n * x // args.slices, n * (x + 1) // args.slices
                    parts.append(orc.search_subset(q, res, off, np.arange(lo, hi, dtype=np.int64), M,
                                                   w.alpha, w.beta, nthreads=args.threads))
                    print(f"[golden] {name} q{i}: slice {x + 1}/{args.slices} "
                          f"({time.time() - t1:.0f}s)", flush=True)
                scores = np.concatenate(parts).astype(np.int32)
            else:
                scores = orc.search(q, res, off, M, w.alpha, w.beta, nthreads=args.threads)
            ts, ti = oracle.topk(scores, K)
            entries[key] = {
                "qlen": len(q), "query_sha256": q_sha,
                "scores_sha256": vector_sha256(scores),
                "top_scores": ts.tolist(), "top_idx": ti.tolist(),
                "max": int(scores.max()), "n_ge_1848": int((scores >= 1848).sum()),
            }
            save(doc, args.out)
            dt = time.time() - t1
            print(f"[golden] {name} q{i} ({len(q)}): {len(q) * int(off[-1]) / dt / 1e9:.2f} "
                  f"GCUPS, {dt:.0f}s, max {int(scores.max())}", flush=True)
    save(doc, args.out)


if __name__ == "__main__":
    main()
