"""GPU parity of the z-step's topic-list upkeep where documents hold about as
many topics as the lists' windows (4 slots per lane, 4G per group of G
lanes): their lists keep crossing between the one-pass window update and the
per-lane loops within a sweep.  Several sweeps per group size, each checked
by the oracle's teacher-forced replay and the exact count rebuild.

Lengths are chosen so that a document of n tokens under uniformly random
topics holds about K (1 - (1 - 1/K)^n) = 4G topics, spread +-30%.
"""
import numpy as np
import pytest

import oracle
from paper_1704_03581_amd import synth
from tests.gpu_helpers import phi_from_gpu, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1704_03581_amd import pulda
else:  # collected on CPU-only hosts, never run there
    pulda = None

K = 1000


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def corpus_near(threshold: int, D: int = 120, seed: int = 41):
    n_star = np.log(1.0 - threshold / K) / np.log(1.0 - 1.0 / K)
    rng = np.random.default_rng(seed)
    lens = np.maximum(1, np.round(n_star * rng.uniform(0.7, 1.3, size=D))).astype(np.int64)
    base = synth.small_random(D=4 * D, V=2000, K=K, mean_len=float(n_star * 1.3), seed=seed, empty_docs=False)
    words = base.words[: int(lens.sum())]
    assert len(words) == lens.sum()
    off = np.zeros(D + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    return synth.Corpus("windows", D, base.V, K, base.alpha, base.beta, off, words.astype(np.int32), None)


def topics_per_doc(off, z):
    return np.array([len(np.unique(z[off[d]:off[d + 1]])) for d in range(len(off) - 1)])


@pytest.mark.parametrize("group", [64, 32, 16, 8])
def test_lists_across_the_window_boundary(group):
    T = 4 * group
    c = corpus_near(T)
    say(f"list windows: group={group} threshold={T} D={c.D} N={c.N}")
    p = pulda.Plan(c.K, c.V, c.D, c.N, alpha=c.alpha, beta=c.beta, seed=29)
    p.upload(c.doc_off, c.words)
    p.set_schedule([0], [group], [64 // group * 4], [1])
    p.init()
    kd0 = topics_per_doc(c.doc_off, p.get_z())
    # documents on both sides of the boundary from the start
    assert (kd0 > T).sum() >= 10 and (kd0 <= T).sum() >= 10, (kd0.min(), kd0.max())
    crossed = 0
    for t in (1, 2, 3):
        z0 = p.get_z()
        p.phi_step(t)
        phi, wt = phi_from_gpu(p.get_phi(), c.K, c.V)
        p.z_step(t)
        z1 = p.get_z()
        r = oracle.replay(c.doc_off, c.words, z0, z1, 29, t, phi, wt, c.K, c.V)
        say(f"  sweep {t}: replay {r}")
        assert r["bad"] == 0, r
        assert r["agree"] >= 0.9999 * c.N
        n_o, _, _ = oracle.counts(c.doc_off, c.words, z1, c.K, c.V, with_m=False)
        assert np.array_equal(p.counts_dense()[0], n_o)
        a, b = topics_per_doc(c.doc_off, z0), topics_per_doc(c.doc_off, z1)
        crossed += int(((a > T) != (b > T)).sum())
    say(f"  documents whose list crossed {T} between sweeps: {crossed}")
    assert crossed > 0
