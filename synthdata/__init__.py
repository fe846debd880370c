"""Seeded synthetic inputs for Smith-Waterman protein database search.

This module only *draws inputs*: residue codes, sequence lengths, a substitution
matrix, query sets, planted homologs and request arrival times.  It contains no
part of the alignment arithmetic, so both the CPU oracle (``oracle/``) and the
GPU library (``paper_1404_4152_amd``) can consume exactly the same bytes while
sharing no code with each other.

The paper evaluates on UniProtKB/TrEMBL 2013_08 and Swiss-Prot queries with
BLOSUM62 and a 10-2k gap penalty (section IV.A).  None of those files are
available, so everything here stands in for them:

* residues: i.i.d. over 20 amino-acid codes drawn from the Robinson & Robinson
  (1991, PNAS 88:8880) background frequencies, quantised to 1/65536;
* lengths: log-normal with sigma 0.75, clipped to the configured range;
* substitution matrix: a seeded "BLOSUM62-style" symmetric int8 matrix built
  from half-bit log-odds of a synthetic conservation model (not BLOSUM62);
* gaps: beta = 12 (open + extension), alpha = 2 (extension), the paper's
  10-2k setting read as open 10, extension 2.

Generator: numpy PCG64 with the seeds given per call.  Every array is
reproducible bit-for-bit from (function, arguments).
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

# 20 standard amino acids, in the order the codes 0..19 use.
AMINO_ACIDS = "ARNDCQEGHILKMFPSTWYV"

# Robinson & Robinson (1991) background frequencies for the letters above.
_RR_FREQ = np.array([
    0.07805, 0.05129, 0.04487, 0.05364, 0.01925, 0.04264, 0.06295, 0.07377,
    0.02199, 0.05142, 0.09019, 0.05744, 0.02243, 0.03856, 0.05203, 0.07120,
    0.05841, 0.01330, 0.03216, 0.06441,
], dtype=np.float64)

ALPHA_DEFAULT = 2    # gap extension
BETA_DEFAULT = 12    # gap open + extension (10-2k)

SEED_DB = 0
SEED_QUERIES = 1
SEED_PLANTED = 2
SEED_ARRIVALS = 3
SEED_MATRIX = 7


def background_frequencies() -> np.ndarray:
    """Background amino-acid frequencies, normalised to sum to 1."""
    return _RR_FREQ / _RR_FREQ.sum()


def _code_table(freqs: np.ndarray) -> np.ndarray:
    """Map a uniform 16-bit draw to a residue code (inverse CDF, 1/65536 grid)."""
    cdf = np.cumsum(freqs / freqs.sum())
    cdf[-1] = 1.0
    grid = (np.arange(65536, dtype=np.float64) + 0.5) / 65536.0
    return np.searchsorted(cdf, grid, side="right").astype(np.uint8)


def random_residues(rng: np.random.Generator, count: int,
                    freqs: np.ndarray | None = None,
                    chunk: int = 1 << 26) -> np.ndarray:
    """``count`` i.i.d. residue codes drawn from ``freqs`` (default background)."""
    if freqs is None:
        freqs = background_frequencies()
    table = _code_table(np.asarray(freqs, dtype=np.float64))
    out = np.empty(count, dtype=np.uint8)
    for lo in range(0, count, chunk):
        hi = min(count, lo + chunk)
        u = rng.integers(0, 65536, size=hi - lo, dtype=np.uint16)
        np.take(table, u, out=out[lo:hi])
    return out


def uniform_residues(rng: np.random.Generator, count: int, alphabet: int) -> np.ndarray:
    """``count`` codes uniform over ``0..alphabet-1`` (small test cases)."""
    return rng.integers(0, alphabet, size=count, dtype=np.uint8) if alphabet > 0 \
        else np.zeros(count, dtype=np.uint8)


def lognormal_lengths(rng: np.random.Generator, n: int, mean: float, lo: int, hi: int,
                      sigma: float = 0.75) -> np.ndarray:
    """Lengths ``clip(rint(exp(N(mu, sigma^2))), lo, hi)`` with the given mean."""
    mu = np.log(mean) - 0.5 * sigma * sigma
    x = np.rint(np.exp(rng.normal(mu, sigma, size=n)))
    return np.clip(x, lo, hi).astype(np.int64)


def blosum_style_matrix(seed: int = SEED_MATRIX, alphabet: int = 20) -> np.ndarray:
    """A seeded symmetric int8 substitution matrix in half-bit log-odds units.

    Construction (documented stand-in for BLOSUM62, not a copy of it): each
    letter ``a`` keeps its identity with probability ``c_a`` drawn from
    U(0.25, 0.5), giving the diagonal ``round(2 log2(c_a / p_a))``; each
    unordered pair ``(a, b)`` gets an exchange ratio ``0.55 * exp(N(0, 0.55))``,
    giving ``round(2 log2(ratio))``.  Scores are clipped to [-4, 11], the range
    of the usual protein matrices.  The expected score of a random pair under
    the background frequencies is negative, which local alignment needs.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    freqs = background_frequencies()
    if alphabet != 20:
        freqs = np.resize(freqs, alphabet)
        freqs = freqs / freqs.sum()
    conserve = rng.uniform(0.25, 0.5, size=alphabet)
    ratio = 0.55 * np.exp(rng.normal(0.0, 0.55, size=(alphabet, alphabet)))
    ratio = np.triu(ratio, 1)
    ratio = ratio + ratio.T
    with np.errstate(divide="ignore"):
        score = np.rint(2.0 * np.log2(np.where(ratio > 0, ratio, 1.0)))
    diag = np.rint(2.0 * np.log2(conserve / freqs))
    score[np.diag_indices(alphabet)] = diag
    score = np.clip(score, -4, 11).astype(np.int8)
    assert (score == score.T).all()
    return score


def random_matrix(rng: np.random.Generator, alphabet: int, lo: int = -6, hi: int = 9,
                  symmetric: bool = False) -> np.ndarray:
    """A random int8 matrix for small test cases (optionally symmetric)."""
    m = rng.integers(lo, hi + 1, size=(alphabet, alphabet)).astype(np.int8)
    if symmetric:
        m = np.triu(m) + np.triu(m, 1).T
    return m.astype(np.int8)


def pack_sequences(seqs: list[np.ndarray]) -> tuple[np.ndarray, np.ndarray]:
    """Concatenate sequences into (residues uint8, offsets int64 of length n+1)."""
    lens = np.array([len(s) for s in seqs], dtype=np.int64)
    offsets = np.zeros(len(seqs) + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    res = np.concatenate([np.asarray(s, dtype=np.uint8) for s in seqs]) if seqs \
        else np.zeros(0, dtype=np.uint8)
    return res, offsets


def make_db(n: int, mean: float, lo: int, hi: int, seed: int = SEED_DB,
            sort: bool = False, uniform_lengths: bool = False) -> tuple[np.ndarray, np.ndarray]:
    """A synthetic protein database: (residues uint8, offsets int64[n+1]).

    Lengths are log-normal (or uniform on [lo, hi] when ``uniform_lengths``);
    residues are i.i.d. background.  ``sort`` orders the sequences by ascending
    length, as the paper's offline index does (section III, stage ii).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if uniform_lengths:
        lens = rng.integers(lo, hi + 1, size=n).astype(np.int64)
    else:
        lens = lognormal_lengths(rng, n, mean, lo, hi)
    if sort:
        lens = np.sort(lens, kind="stable")
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    res = random_residues(rng, int(offsets[-1]))
    return res, offsets


def make_queries(lengths, seed: int = SEED_QUERIES) -> list[np.ndarray]:
    """One background-distributed query per requested length."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [random_residues(rng, int(L)) for L in lengths]


def mutate(rng: np.random.Generator, seq: np.ndarray, identity: float,
           indel_rate: float = 0.02) -> np.ndarray:
    """A homolog of ``seq``: substitutions at rate 1-identity plus short indels."""
    seq = np.asarray(seq, dtype=np.uint8)
    out = seq.copy()
    sub = rng.random(len(seq)) > identity
    out[sub] = random_residues(rng, int(sub.sum()))
    pieces = []
    i = 0
    while i < len(out):
        r = rng.random()
        if r < indel_rate / 2:            # deletion of 1-3 residues
            i += int(rng.integers(1, 4))
            continue
        if r < indel_rate:                # insertion of 1-3 residues
            pieces.append(random_residues(rng, int(rng.integers(1, 4))))
        pieces.append(out[i:i + 1])
        i += 1
    return np.concatenate(pieces) if pieces else np.zeros(0, np.uint8)


def plant_homologs(residues: np.ndarray, offsets: np.ndarray, queries: list[np.ndarray],
                   where: list[int], identity: float = 0.85,
                   seed: int = SEED_PLANTED) -> tuple[np.ndarray, np.ndarray]:
    """Replace DB sequence ``where[k]`` by a homolog of ``queries[k]``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = len(offsets) - 1
    replace = {int(w): mutate(rng, queries[k], identity) for k, w in enumerate(where)}
    seqs = [replace[i] if i in replace else residues[offsets[i]:offsets[i + 1]]
            for i in range(n)]
    return pack_sequences(seqs)


def rebuild_db(residues: np.ndarray, offsets: np.ndarray, replace: dict,
               sort: bool = False) -> tuple[np.ndarray, np.ndarray]:
    """Database with sequence ``i`` replaced by ``replace[i]`` for each key.

    With ``sort`` the result is stably re-sorted by length (the input is
    assumed sorted, so only the replaced sequences move); otherwise every
    sequence keeps its index.  Unchanged sequences are copied as contiguous
    blocks, so this costs one pass over the residues.
    """
    n = len(offsets) - 1
    lens = np.diff(offsets).astype(np.int64)
    keys = np.array(sorted(replace), dtype=np.int64)
    if sort and len(keys):
        keep = np.ones(n, bool)
        keep[keys] = False
        kept = np.flatnonzero(keep)
        src = np.concatenate([kept, -1 - np.arange(len(keys), dtype=np.int64)])
        new_lens = np.concatenate([lens[kept],
                                   np.array([len(replace[int(i)]) for i in keys], np.int64)])
        perm = np.argsort(new_lens, kind="stable")
        src, new_lens = src[perm], new_lens[perm]
    else:
        src = np.arange(n, dtype=np.int64)
        new_lens = lens.copy()
        for j, i in enumerate(keys):
            new_lens[i] = len(replace[int(i)])
            src[i] = -1 - j
    new_off = np.zeros(n + 1, np.int64)
    np.cumsum(new_lens, out=new_off[1:])
    out = np.empty(int(new_off[-1]), np.uint8)
    # Runs of consecutive original indices are copied in one block.
    brk = np.flatnonzero((src[1:] != src[:-1] + 1) | (src[1:] < 0) | (src[:-1] < 0)) + 1
    starts = np.concatenate([[0], brk])
    ends = np.concatenate([brk, [n]])
    for a, b in zip(starts.tolist(), ends.tolist()):
        if src[a] < 0:
            out[new_off[a]:new_off[a + 1]] = replace[int(keys[-1 - src[a]])]
        else:
            o = offsets[src[a]]
            out[new_off[a]:new_off[b]] = residues[o:o + (new_off[b] - new_off[a])]
    return out, new_off


def embed_homologs(residues: np.ndarray, offsets: np.ndarray, queries: list[np.ndarray],
                   identity: float = 0.85, seed: int = SEED_PLANTED
                   ) -> tuple[np.ndarray, np.ndarray, list[int]]:
    """One homolog per query embedded in a random database sequence.

    Sequence ``where[k]`` (distinct, seeded) becomes background flank +
    ``mutate(queries[k], identity)`` + background flank, with its original
    length kept (or the homolog's, if longer): a homologous domain inside a
    longer protein.  Returns (residues, offsets, where).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = len(offsets) - 1
    where = [int(x) for x in rng.choice(n, size=len(queries), replace=False)]
    replace = {}
    for k, i in enumerate(where):
        h = mutate(rng, queries[k], identity)
        total = max(int(offsets[i + 1] - offsets[i]), len(h))
        left = int(rng.integers(0, total - len(h) + 1))
        replace[i] = np.concatenate([random_residues(rng, left), h,
                                     random_residues(rng, total - left - len(h))])
    res, off = rebuild_db(residues, offsets, replace)
    return res, off, where


# Identities of the members of each planted homolog family.
FAMILY_IDENTITIES = (0.45, 0.6, 0.75, 0.85, 0.95)


def plant_families(residues: np.ndarray, offsets: np.ndarray, queries: list[np.ndarray],
                   identities=FAMILY_IDENTITIES, sort: bool = False,
                   seed: int = SEED_PLANTED + 1) -> tuple[np.ndarray, np.ndarray]:
    """A family of whole-length homologs per query, one per identity.

    Each member replaces a distinct random database sequence.  With ``sort``
    the database stays length-sorted (members move to their length's place).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = len(offsets) - 1
    where = rng.choice(n, size=len(queries) * len(identities), replace=False)
    replace = {}
    for k, q in enumerate(queries):
        for f, ident in enumerate(identities):
            replace[int(where[k * len(identities) + f])] = mutate(rng, q, ident)
    return rebuild_db(residues, offsets, replace, sort=sort)


def poisson_arrivals(rate: float, duration: float, seed: int = SEED_ARRIVALS) -> np.ndarray:
    """Open-loop arrival times (seconds) of a Poisson process."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        out.append(t)
    return np.array(out, dtype=np.float64)


def sha256(*arrays: np.ndarray) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


# ---------------------------------------------------------------------------
# Workloads (sizes follow the evaluation's query and database shapes).
# ---------------------------------------------------------------------------
# Lengths of the 20 evaluation queries (section IV.A, 144..5,478 residues).
SCALE_QUERY_LENGTHS = [144, 189, 222, 375, 464, 567, 657, 729, 850, 1000, 1500, 2005,
                       2504, 3005, 3564, 4061, 4548, 4743, 5147, 5478]


@dataclass
class Workload:
    name: str
    n_subjects: int
    mean_len: float
    min_len: int
    max_len: int
    query_lengths: list = field(default_factory=list)
    uniform_lengths: bool = False
    sorted_db: bool = False
    alpha: int = ALPHA_DEFAULT
    beta: int = BETA_DEFAULT
    # Planted homologs: "" none, "embedded" one per query inside a random
    # subject (85% identity), "families" whole-length members per query at
    # FAMILY_IDENTITIES.
    homologs: str = ""

    def db(self):
        res, off = make_db(self.n_subjects, self.mean_len, self.min_len, self.max_len,
                           seed=SEED_DB, sort=self.sorted_db,
                           uniform_lengths=self.uniform_lengths)
        if self.homologs == "embedded":
            res, off, _ = embed_homologs(res, off, self.queries())
        elif self.homologs == "families":
            res, off = plant_families(res, off, self.queries(), sort=self.sorted_db)
        return res, off

    def queries(self):
        return make_queries(self.query_lengths, seed=SEED_QUERIES)

    def matrix(self):
        return blosum_style_matrix()


def _batched_lengths(n=512, lo=50, hi=1500, seed=SEED_QUERIES + 10):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [int(x) for x in rng.integers(lo, hi + 1, size=n)]


WORKLOADS = {
    # 1 query of 144 vs 2,000 subjects (log-normal mean 350, 20..2,000).
    "plain_small": Workload("plain_small", 2000, 350, 20, 2000, [144]),
    # 20 queries (144..5,478) one at a time vs 2M subjects (mean 350, <= 35,000), length-sorted.
    # Each query has a planted family of 5 homologs (45..95% identity).
    "plain_scale": Workload("plain_scale", 2_000_000, 350, 20, 35000,
                            list(SCALE_QUERY_LENGTHS), sorted_db=True, homologs="families"),
    # 8 queries 1,000..5,000 vs 20,000 subjects uniform 5,000..35,000; each
    # query has one 85%-identity homolog embedded in a subject.
    "long_tail": Workload("long_tail", 20000, 20000, 5000, 35000,
                          [int(x) for x in np.rint(np.linspace(1000, 5000, 8))],
                          uniform_lengths=True, homologs="embedded"),
    # 512 queries uniform 50..1,500 vs 500k subjects (mean 350).
    "batched": Workload("batched", 500_000, 350, 20, 35000, _batched_lengths()),
    # Serving DB: 5M subjects (mean 350); queries arrive as a Poisson stream.
    "serving": Workload("serving", 5_000_000, 350, 20, 35000, []),
}


def serving_queries(n: int, seed: int = SEED_QUERIES + 20, mean: float = 400,
                    lo: int = 30, hi: int = 5000) -> list[np.ndarray]:
    """Serving-request queries: log-normal lengths (mean 400, 30..5,000)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lens = lognormal_lengths(rng, n, mean, lo, hi)
    return [random_residues(rng, int(L)) for L in lens]
