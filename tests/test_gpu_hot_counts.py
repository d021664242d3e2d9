"""The count rebuild when the z-step first adds the most frequent words'
increments per block (small K): the rebuilt n_kv and n_k must equal the
counts of the sampled z exactly (Table 1's definition), on both sides of the
topic count where the per-block counters switch off, and after the same plan
takes a second corpus whose frequent words are other word ids.
"""
import numpy as np
import pytest

import oracle
from paper_1704_03581_amd import synth
from tests.gpu_helpers import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1704_03581_amd import pulda
else:
    pulda = None


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


# K = 16: 256 frequent words counted per block; K = 256: 16, the fewest the
# z-step uses; K = 257: none
@pytest.mark.parametrize("K", [16, 256, 257])
def test_counts_with_frequent_word_counters(K):
    c = synth.small_random(D=600, V=2000, K=K, mean_len=150.0, seed=13)
    say(f"frequent-word counters K={K} N={c.N}")
    # the second corpus: the same documents with the vocabulary permuted
    perm = np.random.default_rng(5).permutation(c.V).astype(np.int32)
    p = pulda.Plan(K, c.V, c.D, c.N, alpha=c.alpha, beta=c.beta, seed=3)
    for words in (c.words, perm[c.words]):
        words = np.ascontiguousarray(words, dtype=np.int32)
        p.upload(c.doc_off, words)
        p.init()
        p.sweep(1, 2)
        z = p.get_z()
        n_o, nk_o, _ = oracle.counts(c.doc_off, words, z, K, c.V, with_m=False)
        n_g, nk_g = p.counts_dense()
        assert np.array_equal(n_g, n_o) and np.array_equal(nk_g, nk_o)
