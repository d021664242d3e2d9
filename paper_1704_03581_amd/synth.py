"""Seeded synthetic corpora drawn from the LDA generative model.

This module is the only code shared by the CPU oracle's tests and the GPU
path: it produces inputs and holds none of the sampler's arithmetic.

The generative model is the one of Section 1 (Figure 1, Table 1):
  phi_k ~ Dir(beta-vector), theta_d ~ Dir(alpha 1_K), z ~ Cat(theta_d),
  w ~ Cat(phi_z).
theta_d is integrated out: a document's topic sequence is drawn directly from
its Dirichlet-multinomial marginal by the Polya-urn (Chinese-restaurant)
sequence P(z_j = k | z_<j) = (alpha + m_k) / (K alpha + j), which has the same
law as drawing theta_d and then z iid from it.  That keeps the 8.2M-document
corpus cheap to draw (no D x K gamma matrix).

The configurations mirror the paper's corpora in shape (Table 2) but are
synthetic; the real corpora are not used.
"""
from __future__ import annotations

import dataclasses
import os
from concurrent.futures import ProcessPoolExecutor
from typing import Optional

import numpy as np

CORPUS_SEED_BASE = 170403581

# name -> (index, D, V, K, length model, phi model)
CONFIGS = {
    "tiny": dict(index=0, D=1000, V=5000, K=20, lengths=("poisson", 50.0), phi="symmetric"),
    "small": dict(index=1, D=1500, V=12400, K=100, lengths=("lognormal", 1200.0, 0.329), phi="zipf"),
    "medium": dict(index=2, D=40000, V=28000, K=1000, lengths=("lognormal_tail", 120.0, 0.70, 40, 2000.0, 20000.0),
                   phi="zipf"),
    "large": dict(index=3, D=8_200_000, V=141000, K=1000, lengths=("poisson", 90.0), phi="zipf"),
}
ALPHA = 0.1
BETA = 0.01
ZIPF_EXPONENT = 1.07


@dataclasses.dataclass
class Corpus:
    name: str
    D: int
    V: int
    K: int
    alpha: float
    beta: float
    doc_off: np.ndarray          # int64[D+1]
    words: np.ndarray            # int32[N]
    true_z: Optional[np.ndarray]  # uint16[N] (generating assignments)

    @property
    def N(self) -> int:
        return int(self.doc_off[-1])

    def lengths(self) -> np.ndarray:
        return np.diff(self.doc_off)


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def doc_lengths(model, D: int, rng: np.random.Generator) -> np.ndarray:
    kind = model[0]
    if kind == "poisson":
        return rng.poisson(model[1], size=D).astype(np.int64)
    if kind == "lognormal":
        lens = np.rint(rng.lognormal(np.log(model[1]), model[2], size=D)).astype(np.int64)
        return np.maximum(lens, 1)
    if kind == "lognormal_tail":
        _, median, sigma, n_long, lo, hi = model
        body = np.maximum(np.rint(rng.lognormal(np.log(median), sigma, size=D - n_long)), 1).astype(np.int64)
        j = np.arange(n_long, dtype=np.float64)
        tail = np.rint(lo * (hi / lo) ** (j / (n_long - 1))).astype(np.int64)
        lens = np.concatenate([body, tail])
        return lens[rng.permutation(D)]
    raise ValueError(kind)


def zipf_base_measure(V: int, rng: np.random.Generator) -> np.ndarray:
    """F0 over word ids: Zipf(1.07) over ranks, ranks scattered by a permutation."""
    ranks = np.arange(V, dtype=np.float64)
    f = (ranks + 1.0) ** (-ZIPF_EXPONENT)
    f /= f.sum()
    perm = rng.permutation(V)      # word id perm[r] has rank r
    out = np.empty(V)
    out[perm] = f
    return out


def true_phi(cfg: dict, seed: int) -> np.ndarray:
    """Generating topic-word matrix (K x V, float64, rows sum to 1)."""
    K, V = cfg["K"], cfg["V"]
    rng = _rng(seed, 1)
    if cfg["phi"] == "symmetric":
        conc = np.full(V, BETA)
    else:
        conc = BETA * V * zipf_base_measure(V, rng)
    phi = np.empty((K, V))
    for k in range(K):
        g = rng.standard_gamma(conc)
        phi[k] = g / g.sum()
    return phi


def _topics_polya(lens: np.ndarray, K: int, alpha: float, rng: np.random.Generator) -> np.ndarray:
    """Topic sequences of all documents by the Polya-urn draw, vectorised over documents."""
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    z = np.empty(int(off[-1]), dtype=np.uint16)
    order = np.argsort(-lens, kind="stable")      # longest first: active docs are a prefix
    sorted_lens = lens[order]
    starts = off[:-1][order]
    maxlen = int(sorted_lens[0]) if len(lens) else 0
    n_active = len(lens)
    Ka = K * alpha
    for j in range(maxlen):
        while n_active > 0 and sorted_lens[n_active - 1] <= j:
            n_active -= 1
        st = starts[:n_active]
        pos = st + j
        if j == 0:
            z[pos] = rng.integers(0, K, size=n_active)
            continue
        fresh = rng.random(n_active) < Ka / (Ka + j)
        nf = int(fresh.sum())
        z[pos[fresh]] = rng.integers(0, K, size=nf)
        cp = ~fresh
        src = st[cp] + rng.integers(0, j, size=n_active - nf)
        z[pos[cp]] = z[src]
    return z


def _words_given_topics(z: np.ndarray, cdf: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    K, V = cdf.shape
    words = np.empty(len(z), dtype=np.int32)
    order = np.argsort(z, kind="stable")
    counts = np.bincount(z, minlength=K)
    start = 0
    for k in range(K):
        c = int(counts[k])
        if c:
            u = rng.random(c)
            w = np.searchsorted(cdf[k], u, side="right")
            np.minimum(w, V - 1, out=w)
            words[order[start:start + c]] = w
            start += c
    return words


_SHARD_CDF = None


def _shard_worker(args):
    lens, K, alpha, seed, shard = args
    rng = _rng(seed, 2, shard)
    z = _topics_polya(lens, K, alpha, rng)
    w = _words_given_topics(z, _SHARD_CDF, rng)
    return w, z


def generate(name: str, seed: Optional[int] = None, workers: Optional[int] = None,
             keep_true_z: bool = True) -> Corpus:
    """Draw the named synthetic corpus.  Deterministic in (name, seed)."""
    global _SHARD_CDF
    cfg = CONFIGS[name]
    if seed is None:
        seed = CORPUS_SEED_BASE + cfg["index"]
    D, V, K = cfg["D"], cfg["V"], cfg["K"]
    lens = doc_lengths(cfg["lengths"], D, _rng(seed, 0))
    phi = true_phi(cfg, seed)
    cdf = np.cumsum(phi, axis=1)
    cdf /= cdf[:, -1:]
    del phi
    # fixed sharding by document ranges; each shard has its own stream, so the
    # corpus does not depend on the number of worker processes
    shard_docs = 262144
    shards = [(lens[s:s + shard_docs], K, ALPHA, seed, i)
              for i, s in enumerate(range(0, D, shard_docs))]
    _SHARD_CDF = cdf
    if workers is None:
        workers = min(16, os.cpu_count() or 1, len(shards))
    if workers > 1 and len(shards) > 1:
        import multiprocessing as mp
        with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
            parts = list(ex.map(_shard_worker, shards))
    else:
        parts = [_shard_worker(s) for s in shards]
    _SHARD_CDF = None
    words = np.concatenate([p[0] for p in parts]) if parts else np.zeros(0, np.int32)
    z = np.concatenate([p[1] for p in parts]) if (parts and keep_true_z) else None
    off = np.zeros(D + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    return Corpus(name, D, V, K, ALPHA, BETA, off, words, z)


def save(c: Corpus, path: str) -> None:
    """Write a corpus as a plain .npz (no pickled objects)."""
    np.savez(path, name=np.array(c.name), shape=np.array([c.D, c.V, c.K], np.int64),
             prior=np.array([c.alpha, c.beta]), doc_off=c.doc_off, words=c.words)


def load(path: str) -> Corpus:
    with np.load(path, allow_pickle=False) as f:
        D, V, K = (int(x) for x in f["shape"])
        alpha, beta = (float(x) for x in f["prior"])
        return Corpus(str(f["name"]), D, V, K, alpha, beta, f["doc_off"], f["words"], None)


def restrict(c: Corpus, min_count: int = 0, max_vocab: Optional[int] = None, doc_fraction: float = 1.0,
             max_len: Optional[int] = None) -> Corpus:
    """The preprocessing that the paper's scaling study varies (Section 4):
    keep the first doc_fraction of the documents (and, with max_len, only
    those of at most max_len tokens), drop the words that occur
    fewer than min_count times in them (the rare-word limit), keep at most
    max_vocab of the rest, most frequent first (the paper ranks by TF-IDF,
    here by frequency), and renumber the kept words 0 .. V'-1 in their
    original order.  Tokens of dropped words leave their documents."""
    D = max(1, int(round(c.D * doc_fraction)))
    off = c.doc_off[: D + 1]
    w = c.words[: off[-1]]
    if max_len is not None:
        lens = np.diff(off)
        ok = lens <= max_len
        w = w[np.repeat(ok, lens)]
        D = int(ok.sum())
        off = np.zeros(D + 1, np.int64)
        np.cumsum(lens[ok], out=off[1:])
    cnt = np.bincount(w, minlength=c.V)
    keep = cnt >= max(min_count, 1)
    if max_vocab is not None and keep.sum() > max_vocab:
        order = np.argsort(-cnt, kind="stable")
        top = np.zeros(c.V, bool)
        top[order[:max_vocab]] = True
        keep &= top
    new_id = np.full(c.V, -1, np.int64)
    new_id[keep] = np.arange(int(keep.sum()))
    mapped = new_id[w]
    kept_tok = mapped >= 0
    doc_of = np.repeat(np.arange(D), np.diff(off))
    lens = np.bincount(doc_of[kept_tok], minlength=D)
    new_off = np.zeros(D + 1, np.int64)
    np.cumsum(lens, out=new_off[1:])
    return Corpus(f"{c.name}/min{min_count}/V{max_vocab}/f{doc_fraction}/L{max_len}", D, int(keep.sum()), c.K, c.alpha,
                  c.beta, new_off, mapped[kept_tok].astype(np.int32), None)


def small_random(D: int, V: int, K: int, mean_len: float, seed: int, zipf: bool = True,
                 empty_docs: bool = True) -> Corpus:
    """A small corpus of arbitrary shape for tests (Poisson lengths)."""
    rng = _rng(seed, 7)
    lens = rng.poisson(mean_len, size=D).astype(np.int64)
    if not empty_docs:
        lens = np.maximum(lens, 1)
    cfg = dict(K=K, V=V, phi="zipf" if zipf else "symmetric")
    phi = true_phi(cfg, seed)
    cdf = np.cumsum(phi, axis=1)
    cdf /= cdf[:, -1:]
    z = _topics_polya(lens, K, ALPHA, rng) if lens.sum() else np.zeros(0, np.uint16)
    words = _words_given_topics(z, cdf, rng) if len(z) else np.zeros(0, np.int32)
    off = np.zeros(D + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    return Corpus("custom", D, V, K, ALPHA, BETA, off, words, z)


def topic_word_counts_draw(name: str, seed: Optional[int] = None) -> np.ndarray:
    """Topic-word counts n (K x V int32) of the named corpus's shape, drawn directly.

    Used to build a trained-looking sparse Phi for fold-in serving without
    materialising the 738M-token corpus: the topic totals follow the corpus's
    expected mixture and each row is Multinomial(n_k., phi_k).
    """
    cfg = CONFIGS[name]
    if seed is None:
        seed = CORPUS_SEED_BASE + cfg["index"]
    rng = _rng(seed, 3)
    lens = doc_lengths(cfg["lengths"], cfg["D"], _rng(seed, 0))
    N = int(lens.sum())
    K = cfg["K"]
    phi = true_phi(cfg, seed)
    totals = rng.multinomial(N, rng.dirichlet(np.full(K, 1.0)))
    n = np.empty((K, cfg["V"]), dtype=np.int32)
    for k in range(K):
        n[k] = rng.multinomial(int(totals[k]), phi[k])
    return n


def foldin_requests(n_requests: int, seed: int, base: str = "large",
                    min_len: int = 10, max_len: int = 5000) -> list:
    """New documents for fold-in: lengths LogNormal(ln 200, 1.0) resampled into
    [min_len, max_len]; words from the base corpus's generating Phi with
    theta ~ Dir(alpha)."""
    cfg = CONFIGS[base]
    rng = _rng(seed, 4)
    lens = np.empty(n_requests, dtype=np.int64)
    filled = 0
    while filled < n_requests:
        cand = np.rint(rng.lognormal(np.log(200.0), 1.0, size=2 * (n_requests - filled) + 16)).astype(np.int64)
        cand = cand[(cand >= min_len) & (cand <= max_len)]
        take = min(len(cand), n_requests - filled)
        lens[filled:filled + take] = cand[:take]
        filled += take
    phi = true_phi(cfg, CORPUS_SEED_BASE + cfg["index"])
    cdf = np.cumsum(phi, axis=1)
    cdf /= cdf[:, -1:]
    K = cfg["K"]
    z = _topics_polya(lens, K, ALPHA, rng)
    words = _words_given_topics(z, cdf, rng)
    off = np.zeros(n_requests + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    return [words[off[i]:off[i + 1]].copy() for i in range(n_requests)]
