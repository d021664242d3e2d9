"""The corpus restrictions of the scaling study (CPU only)."""
import numpy as np

from paper_1704_03581_amd import synth


def test_restrict_keeps_order_counts_and_limits():
    c = synth.small_random(D=300, V=700, K=20, mean_len=40.0, seed=8)
    for g in [dict(min_count=5), dict(max_vocab=120), dict(doc_fraction=0.4), dict(min_count=2, max_vocab=60)]:
        r = synth.restrict(c, **g)
        D = max(1, int(round(c.D * g.get("doc_fraction", 1.0))))
        assert r.D == D and r.doc_off[0] == 0 and r.doc_off[-1] == len(r.words)
        w0 = c.words[: c.doc_off[D]]
        cnt0 = np.bincount(w0, minlength=c.V)
        kept = cnt0 >= max(g.get("min_count", 0), 1)
        if "max_vocab" in g and kept.sum() > g["max_vocab"]:
            kept &= np.isin(np.arange(c.V), np.argsort(-cnt0, kind="stable")[: g["max_vocab"]])
        ids = np.nonzero(kept)[0]
        assert r.V == len(ids)
        # each document keeps its kept tokens, in order, renumbered by rank of id
        for d in range(0, D, 17):
            doc = c.words[c.doc_off[d]:c.doc_off[d + 1]]
            exp = np.searchsorted(ids, doc[np.isin(doc, ids)])
            assert np.array_equal(r.words[r.doc_off[d]:r.doc_off[d + 1]], exp)
        assert np.bincount(r.words, minlength=r.V).min() >= max(g.get("min_count", 0), 1)


def test_restrict_max_len():
    c = synth.small_random(D=100, V=300, K=10, mean_len=40.0, seed=9)
    r = synth.restrict(c, max_len=40)
    lens = np.diff(c.doc_off)
    assert r.D == int((lens <= 40).sum()) and np.diff(r.doc_off).max() <= 40
    assert r.N == int(lens[lens <= 40].sum())
