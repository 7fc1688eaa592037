"""Seeded synthetic inputs for the alignment path.

This module only draws sequences and builds input arrays; it holds none of
the alignment arithmetic.  It is the one module that both the GPU-side tests
and benchmark and the oracle-side checks use for inputs.

Symbols are small integer codes.  DNA uses A=0, C=1, G=2, T=3.  Proteins use
24 codes (20 residues plus 4 ambiguity/stop codes that the generators never
emit).  Scoring matrices are row-major n x n int8, indexed [query][reference].

The five workloads follow the problem sizes of the paper's own experiments
(short reads against windows, a read against a multi-megabase reference,
protein one-against-many search, many read/window pairs, and a request
stream).  They are synthetic stand-ins for the paper's datasets, which are not
available here; the recipe of each is stated in its docstring.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 12086350
DNA = 4
N_PROTEIN = 24


def rng_for(k: int) -> np.random.Generator:
    """The generator of workload k (1-based)."""
    return np.random.Generator(np.random.PCG64(SEED_BASE + k))


def dna_matrix(match: int = 2, mismatch: int = -2, n: int = DNA) -> np.ndarray:
    m = np.full((n, n), mismatch, dtype=np.int8)
    np.fill_diagonal(m, match)
    return m


def protein_matrix_standin(seed: int = SEED_BASE + 300) -> np.ndarray:
    """A labelled STAND-IN for BLOSUM62 (no such table is available here).

    Symmetric 24 x 24 int8 with a dominant diagonal in [4, 11] and
    off-diagonal entries drawn from [-4, 3], then lowered by one at a time
    (never below -4) until the expected score of two residues drawn from the
    background frequencies (background_standin) is at most -1, as for
    BLOSUM-type matrices (a local alignment of unrelated sequences then stays
    short; with a positive expectation every target would align end to end).
    The last four codes (ambiguity/stop) score -1 against residues and 1
    against themselves.
    """
    g = np.random.Generator(np.random.PCG64(seed))
    m = g.integers(-4, 4, size=(N_PROTEIN, N_PROTEIN)).astype(np.int64)
    m = np.triu(m) + np.triu(m, 1).T
    np.fill_diagonal(m, g.integers(4, 12, size=N_PROTEIN))
    f = background_standin()[:20]
    off = ~np.eye(20, dtype=bool)
    while float(f @ m[:20, :20] @ f) > -1.0:
        sub = m[:20, :20]
        sub[off] = np.maximum(sub[off] - 1, -4)
        m[:20, :20] = sub
    m[20:, :] = -1
    m[:, 20:] = -1
    for k in range(20, N_PROTEIN):
        m[k, k] = 1
    return m.astype(np.int8)


def background_standin(seed: int = SEED_BASE + 301) -> np.ndarray:
    """A labelled STAND-IN for background amino-acid frequencies (20 residues,
    skewed like real proteomes: between about 1% and 10%)."""
    g = np.random.Generator(np.random.PCG64(seed))
    w = g.gamma(4.0, 1.0, size=20)
    w = w / w.sum()
    f = np.zeros(N_PROTEIN)
    f[:20] = w
    return f


@dataclass
class Batch:
    """Pairs of (query, reference) over concatenated code arrays."""
    name: str
    matrix: np.ndarray
    gap_open: int
    gap_extend: int
    qcat: np.ndarray
    qoff: np.ndarray
    rcat: np.ndarray
    roff: np.ndarray
    pair_q: np.ndarray
    pair_r: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def npairs(self) -> int:
        return int(len(self.pair_q))

    def qlen(self):
        return (self.qoff[1:] - self.qoff[:-1])[self.pair_q]

    def rlen(self):
        return (self.roff[1:] - self.roff[:-1])[self.pair_r]

    def cells(self) -> int:
        return int(np.sum(self.qlen().astype(np.int64) * self.rlen().astype(np.int64)))

    def query(self, p: int) -> np.ndarray:
        qi = self.pair_q[p]
        return self.qcat[self.qoff[qi]:self.qoff[qi + 1]]

    def ref(self, p: int) -> np.ndarray:
        ri = self.pair_r[p]
        return self.rcat[self.roff[ri]:self.roff[ri + 1]]

    def subset(self, idx) -> "Batch":
        """A batch of the selected pairs (sequences re-packed)."""
        idx = np.asarray(idx, dtype=np.int64)
        qs = [self.query(int(p)) for p in idx]
        rs = [self.ref(int(p)) for p in idx]
        return from_lists(self.name + "-subset", self.matrix, self.gap_open, self.gap_extend,
                          qs, rs, dict(self.meta))


def concat(seqs):
    lens = np.array([len(s) for s in seqs], dtype=np.int64)
    off = np.zeros(len(seqs) + 1, dtype=np.int64)
    if len(seqs):
        off[1:] = np.cumsum(lens)
    cat = np.concatenate([np.asarray(s, dtype=np.int8) for s in seqs]) if len(seqs) else \
        np.zeros(0, dtype=np.int8)
    return cat.astype(np.int8), off


def from_lists(name, matrix, o, e, queries, refs, meta=None) -> Batch:
    """One pair per (queries[k], refs[k])."""
    qcat, qoff = concat(queries)
    rcat, roff = concat(refs)
    idx = np.arange(len(queries), dtype=np.int64)
    return Batch(name, np.asarray(matrix, dtype=np.int8), int(o), int(e), qcat, qoff, rcat, roff,
                 idx, idx.copy(), meta or {})


# ---------------------------------------------------------------------------
# sequence mutation (vectorised over many sequences at once)
# ---------------------------------------------------------------------------
def mutate_many(g: np.random.Generator, cat: np.ndarray, off: np.ndarray,
                sub_rate, ins_rate, del_rate, max_indel: int, alphabet: int = DNA):
    """Apply per-base events to every sequence of (cat, off).

    Each base independently: substitution (to one of the other symbols,
    uniformly) with probability sub_rate; insertion after it with ins_rate;
    deletion starting at it with del_rate.  Indel lengths are uniform in
    [1, max_indel].  Rates may be scalars or one value per sequence.
    Returns (new_cat, new_off).
    """
    nseq = len(off) - 1
    lens = off[1:] - off[:-1]
    sid = np.repeat(np.arange(nseq), lens)
    per = lambda x: (np.full(nseq, x) if np.isscalar(x) else np.asarray(x))[sid]
    ps, pi, pd = per(sub_rate), per(ins_rate), per(del_rate)
    u = g.random(len(cat))
    sub = u < ps
    ins = (u >= ps) & (u < ps + pi)
    dele = (u >= ps + pi) & (u < ps + pi + pd)
    out = cat.astype(np.int16).copy()
    shift = g.integers(1, alphabet, size=len(cat))
    out[sub] = (out[sub] + shift[sub]) % alphabet
    keep = np.ones(len(cat), dtype=bool)
    dl = g.integers(1, max_indel + 1, size=len(cat))
    starts = np.nonzero(dele)[0]
    for t in range(max_indel):
        p = starts[dl[starts] > t] + t
        p = p[p < len(cat)]
        p = p[sid[p] == sid[p - t]]
        keep[p] = False
    il = np.where(ins, g.integers(1, max_indel + 1, size=len(cat)), 0)
    counts = keep.astype(np.int64) + np.where(keep, il, 0)
    rep = np.repeat(out, counts)
    # the first copy of each kept base keeps its symbol; the rest are inserted
    first = np.zeros(len(rep), dtype=bool)
    pos = np.cumsum(counts) - counts
    first[pos[counts > 0]] = True
    rep[~first] = g.integers(0, alphabet, size=int((~first).sum()))
    newlens = np.add.reduceat(counts, off[:-1]) if len(cat) else np.zeros(nseq, np.int64)
    newlens = np.where(lens > 0, newlens, 0)
    noff = np.zeros(nseq + 1, dtype=np.int64)
    noff[1:] = np.cumsum(newlens)
    return rep.astype(np.int8), noff


def random_dna(g, n):
    return g.integers(0, DNA, size=n).astype(np.int8)


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------
def config1(seed_k: int = 1) -> Batch:
    """Single DNA pair: a 150-nt read against a 2,000-nt window.

    Window i.i.d. uniform ACGT; the read is a window substring at a uniform
    offset with 2% substitutions and 0.5% indels (insertion:deletion 1:1,
    length uniform 1-3).  Scoring +2/-2, gap open 3, extend 1."""
    g = rng_for(seed_k)
    win = random_dna(g, 2000)
    p = int(g.integers(0, 2000 - 150 + 1))
    src = win[p:p + 150]
    rc, roff = mutate_many(g, src, np.array([0, 150]), 0.02, 0.0025, 0.0025, 3)
    return from_lists("c1-single-dna", dna_matrix(), 3, 1, [rc], [win],
                      {"locus": p})


def config2(seed_k: int = 2, ref_len: int = 5_000_000, read_len: int = 1000) -> Batch:
    """Single long-reference pair: a 1,000-nt read against a 5,000,000-nt
    i.i.d. ACGT reference.  The read copies a uniform locus with 1%
    substitutions and 0.3% indels (length 1-3).  Three near-copies of the
    locus's source segment (5% substitutions, no indels) are planted at
    uniform loci at least 10 kb from the locus and from each other."""
    g = rng_for(seed_k)
    ref = random_dna(g, ref_len)
    locus = int(g.integers(0, ref_len - read_len))
    src = ref[locus:locus + read_len].copy()
    read, _ = mutate_many(g, src, np.array([0, read_len]), 0.01, 0.0015, 0.0015, 3)
    placed = [locus]
    copies = []
    while len(copies) < 3:
        c = int(g.integers(0, ref_len - read_len))
        if all(abs(c - x) >= 10_000 for x in placed):
            nc, _ = mutate_many(g, src, np.array([0, read_len]), 0.05, 0.0, 0.0, 1)
            ref[c:c + read_len] = nc
            placed.append(c)
            copies.append(c)
    return from_lists("c2-long-ref", dna_matrix(), 3, 1, [read], [ref],
                      {"locus": locus, "copies": copies})


def config3(seed_k: int = 3, ntargets: int = 100_000, qlen: int = 300) -> Batch:
    """Protein one-against-many: a 300-aa query against 100,000 targets of
    length round(LogNormal(ln 300, 0.6)) clipped to [50, 5000], residues i.i.d.
    from background frequencies.  Gap open 11, extend 1.  The matrix and the
    frequencies are labelled stand-ins (see protein_matrix_standin)."""
    g = rng_for(seed_k)
    freq = background_standin()
    query = g.choice(N_PROTEIN, size=qlen, p=freq).astype(np.int8)
    lens = np.clip(np.round(g.lognormal(np.log(300.0), 0.6, size=ntargets)), 50, 5000)
    lens = lens.astype(np.int64)
    rcat = g.choice(N_PROTEIN, size=int(lens.sum()), p=freq).astype(np.int8)
    roff = np.zeros(ntargets + 1, dtype=np.int64)
    roff[1:] = np.cumsum(lens)
    qoff = np.array([0, qlen], dtype=np.int64)
    return Batch("c3-protein-search", protein_matrix_standin(), 11, 1, query, qoff, rcat, roff,
                 np.zeros(ntargets, dtype=np.int64), np.arange(ntargets, dtype=np.int64),
                 {"matrix": "stand-in", "frequencies": "stand-in"})


def config4(seed_k: int = 4, npairs: int = 1_000_000) -> Batch:
    """Batched uneven DNA: read/window pairs.  Source length uniform
    100-250; window = source plus a uniform 0-400 nt ACGT flank split
    uniformly left/right.  Per-read substitution rate uniform in [1%, 3%],
    0.5% indels (length 1-3); 10% of reads are replaced by i.i.d. random reads
    of the same length (no true hit).  Scoring +2/-2, gap open 3, extend 1."""
    g = rng_for(seed_k)
    slen = g.integers(100, 251, size=npairs).astype(np.int64)
    flank = g.integers(0, 401, size=npairs).astype(np.int64)
    left = (g.random(npairs) * (flank + 1)).astype(np.int64)
    left = np.minimum(left, flank)
    right = flank - left
    soff = np.zeros(npairs + 1, dtype=np.int64)
    soff[1:] = np.cumsum(slen)
    src = random_dna(g, int(soff[-1]))
    subr = g.uniform(0.01, 0.03, size=npairs)
    qcat, qoff = mutate_many(g, src, soff, subr, 0.0025, 0.0025, 3)
    # random reads (10%)
    rnd = g.random(npairs) < 0.10
    if rnd.any():
        qlens = qoff[1:] - qoff[:-1]
        qid = np.repeat(np.arange(npairs), qlens)
        mask = rnd[qid]
        qcat = qcat.copy()
        qcat[mask] = random_dna(g, int(mask.sum()))
    # windows: left flank + source + right flank
    wlen = slen + flank
    roff = np.zeros(npairs + 1, dtype=np.int64)
    roff[1:] = np.cumsum(wlen)
    rcat = random_dna(g, int(roff[-1]))
    # copy each source into its window at offset `left`
    wid = np.repeat(np.arange(npairs), slen)
    within = np.arange(int(soff[-1])) - np.repeat(soff[:-1], slen)
    rcat[roff[:-1][wid] + left[wid] + within] = src
    idx = np.arange(npairs, dtype=np.int64)
    return Batch("c4-batched-dna", dna_matrix(), 3, 1, qcat, qoff, rcat, roff, idx, idx.copy(),
                 {"random_read": rnd, "left": left})


@dataclass
class RequestPool:
    """Request pool and arrival schedule of the serving workload."""
    batch: Batch                # one pair per request in the pool
    is_long: np.ndarray         # bool per pool entry
    arrivals: np.ndarray        # arrival times in seconds (sorted)
    which: np.ndarray           # pool index of each arrival
    rate: float


def config5_pool(seed_k: int = 5, n_short: int = 50_000, n_long: int = 1_000) -> Batch:
    """Serving pool: short requests (150-nt read vs 1,000-nt window, 2% error)
    and long ones (10,000-nt read vs 20,000-nt window, 10% error), with
    substitution:insertion:deletion = 2:1:1 and indel length 1."""
    g = rng_for(seed_k)

    def make(n, rl, wl, err):
        flank = wl - rl
        src_off = np.arange(n + 1, dtype=np.int64) * rl
        src = random_dna(g, n * rl)
        reads, roffs = mutate_many(g, src, src_off, err / 2, err / 4, err / 4, 1)
        left = g.integers(0, flank + 1, size=n)
        win = random_dna(g, n * wl).reshape(n, wl)
        s2 = src.reshape(n, rl)
        for k in range(n):
            win[k, left[k]:left[k] + rl] = s2[k]
        qs = [reads[roffs[k]:roffs[k + 1]] for k in range(n)]
        return qs, list(win)

    qs, ws = make(n_short, 150, 1000, 0.02)
    ql, wl = make(n_long, 10_000, 20_000, 0.10)
    b = from_lists("c5-serving-pool", dna_matrix(), 3, 1, qs + ql, ws + wl)
    b.meta["is_long"] = np.array([False] * n_short + [True] * n_long)
    return b


def all_vs_all(n_reads: int = 4000, read_len: int = 70, region_len: int = 1500,
               sub_rate: float = 0.01, seed_k: int = 6) -> Batch:
    """All-vs-all overlap of short reads from one region: n_reads reads of
    read_len nt drawn at uniform offsets of an i.i.d. region_len-nt ACGT
    region, each with sub_rate substitutions per base; every pair i < j is
    aligned (+2/-2, gap open 3, extend 1).  Stands in for a read-overlap graph
    over reads of one genomic locus: no real read set is available.  The
    reads are stored once and serve as queries and references."""
    g = rng_for(seed_k)
    region = random_dna(g, region_len)
    starts = g.integers(0, region_len - read_len + 1, size=n_reads)
    src = np.concatenate([region[s:s + read_len] for s in starts])
    off = np.arange(n_reads + 1, dtype=np.int64) * read_len
    reads, roff = mutate_many(g, src, off, sub_rate, 0.0, 0.0, 1)
    iu, ju = np.triu_indices(n_reads, k=1)
    return Batch(f"all-vs-all-{n_reads}x{read_len}", dna_matrix(), 3, 1, reads, roff,
                 reads, roff, iu.astype(np.int64), ju.astype(np.int64),
                 {"starts": starts})


def poisson_schedule(g: np.random.Generator, rate: float, duration: float, pool_size: int,
                     is_long: np.ndarray | None = None, long_frac: float = 0.10):
    """Open-loop Poisson arrivals over `duration` seconds; each arrival draws a
    pool entry (long with probability long_frac when is_long is given)."""
    n = int(g.poisson(rate * duration))
    t = np.sort(g.uniform(0.0, duration, size=n))
    if is_long is None:
        which = g.integers(0, pool_size, size=n)
    else:
        longs = np.nonzero(is_long)[0]
        shorts = np.nonzero(~is_long)[0]
        pick_long = g.random(n) < long_frac
        which = np.where(pick_long, longs[g.integers(0, len(longs), size=n)],
                         shorts[g.integers(0, len(shorts), size=n)])
    return t, which


def random_pairs(seed: int, npairs: int, qlen_range, rlen_range, alphabet: int = DNA,
                 matrix=None, o: int = 3, e: int = 1, planted: float = 0.5) -> Batch:
    """Small random pairs for parity tests: lengths uniform in the ranges;
    a fraction of the queries are mutated substrings of their references."""
    g = np.random.Generator(np.random.PCG64(seed))
    qs, rs = [], []
    for _ in range(npairs):
        lq = int(g.integers(qlen_range[0], qlen_range[1] + 1))
        lr = int(g.integers(rlen_range[0], rlen_range[1] + 1))
        r = g.integers(0, alphabet, size=lr).astype(np.int8)
        if g.random() < planted and lr > 0 and lq > 0:
            ln = min(lq, lr)
            p = int(g.integers(0, lr - ln + 1))
            src = r[p:p + ln]
            q, _ = mutate_many(g, src, np.array([0, ln]), 0.05, 0.02, 0.02, 3, alphabet)
            if len(q) == 0:
                q = g.integers(0, alphabet, size=max(lq, 1)).astype(np.int8)
        else:
            q = g.integers(0, alphabet, size=max(lq, 1)).astype(np.int8)
        qs.append(q)
        rs.append(r)
    if matrix is None:
        matrix = dna_matrix(n=alphabet) if alphabet <= 8 else protein_matrix_standin()
    return from_lists(f"random-{seed}", matrix, o, e, qs, rs)
