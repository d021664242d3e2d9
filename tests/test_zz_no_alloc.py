"""The held-out estimate's entry point without a workspace
(pulda_heldout_loglik_noalloc), called through the C ABI, against the
entry point with a caller workspace, whose parity with the oracle the
held-out tests establish.  Both run the same kernels on the same inputs, so
estimates, kept counts and every particle's normalisers must be equal bit
for bit: two calls in a row, the second with a smaller input (so nothing
may carry over from the first call's scratch), then a call too large for the
library's scratch, which must be refused before any launch.
"""
import numpy as np
import pytest

from paper_1704_03581_amd import synth
from tests.gpu_helpers import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1704_03581_amd import pulda
else:
    pulda = None


def _docs(V, lens, seed):
    rng = np.random.default_rng(seed)
    return [rng.integers(0, V + 3, n).astype(np.int32) for n in lens]   # a few ids >= V: dropped


def _same(p, docs, R, group, seed):
    a = p.heldout_loglik(docs, req=np.arange(len(docs)) + 7, particles=R, group=group, seed=seed, want_Z=True)
    b = p.heldout_loglik(docs, req=np.arange(len(docs)) + 7, particles=R, group=group, seed=seed, want_Z=True,
                         noalloc=True)
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[0].view(np.uint64), b[0].view(np.uint64))
    for za, zb in zip(a[2], b[2]):
        assert np.array_equal(za.view(np.uint64), zb.view(np.uint64))
    return a


def test_noalloc_heldout_equals_workspace_entry_point():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = synth.small_random(D=200, V=2000, K=200, mean_len=120.0, seed=19)
    p = pulda.Plan(c.K, c.V, c.D, c.N, alpha=c.alpha, beta=c.beta, seed=5)
    p.upload(c.doc_off, c.words)
    p.init()
    p.sweep(1, 3, want_ll=False)
    p.phi_step(4)
    big = _docs(c.V, [0, 1, 3, 40, 77, 150, 230, 12, 5, 64] * 4, seed=1)
    small = _docs(c.V, [2, 9, 30, 17], seed=2)
    R = 8
    n_big = sum(len(d) for d in big)
    say(f"no-alloc held-out: {len(big)} documents, {n_big} tokens, then {len(small)} documents")
    ll, kept, _ = _same(p, big, R, 32, 3)
    assert np.all(np.isfinite(ll[kept > 0]))
    _same(p, small, R, 32, 4)
    _same(p, small, R, 64, 4)
    # a call whose scratch exceeds the library's array is refused on the host
    n_tok = pulda.HELDOUT_NOALLOC_SCRATCH_BYTES // (14 * R) + 1000
    long_docs = [np.zeros(60000, np.int32) for _ in range(n_tok // 60000 + 1)]
    with pytest.raises(pulda.PuldaError) as e:
        p.heldout_loglik(long_docs, particles=R, noalloc=True)
    assert e.value.status == pulda.ERR_NO_MEMORY
    say(f"  refused: {e.value}")
    # and the scratch still serves the next call
    _same(p, small, R, 32, 4)
