"""GPU parity of the held-out log-likelihood (left-to-right estimate),
called through the C ABI, against the CPU oracle.

Each particle's draws follow the token conditional of the z-step, drawn
from the same Philox counters on both sides, so the particles' topic paths
agree draw for draw; Z_n = sigma_a + sigma_b differs only by the fp64
summation order of sigma_b (a group scan on the GPU, a sequential sum in the
oracle): at most (K + 1) * 2^-52 relative, and the estimate, a sum of logs of
particle means of Z, as much per step.  The tests allow 1e-12 relative on Z
and on the estimate.
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
else:
    pulda = None

RTOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _model(c, seed, method="polya_urn"):
    p = pulda.Plan(c.K, c.V, c.D, c.N, alpha=c.alpha, beta=c.beta, seed=seed)
    p.upload(c.doc_off, c.words)
    p.set_phi_method(method)
    p.init()
    p.sweep(1, 3, want_ll=False)
    p.phi_step(4)
    return p


def _docs(V, lens, seed):
    rng = np.random.default_rng(seed)
    docs = [rng.integers(0, V, n).astype(np.int32) for n in lens]
    return docs


def _compare(p, c, docs, R, group, seed):
    ll, kept, Zs = p.heldout_loglik(docs, req=np.arange(len(docs)) + 100, particles=R, group=group, seed=seed,
                                    want_Z=True)
    phi, wt = phi_from_gpu(p.get_phi(), c.K, c.V)
    alpha = np.broadcast_to(c.alpha, (c.K,))
    worst = 0.0
    for d, w in enumerate(docs):
        ll_o, kept_o, Z_o = oracle.heldout_ltr(phi, wt, alpha, seed, 100 + d, w, R, want_Z=True)
        assert kept[d] == kept_o, d
        if kept_o == 0:
            assert ll[d] == 0.0
            continue
        rel = np.abs(Zs[d] - Z_o) / Z_o
        worst = max(worst, float(rel.max()))
        assert rel.max() <= RTOL, (d, rel.max())
        assert abs(ll[d] - ll_o) <= RTOL * abs(ll_o), (d, ll[d], ll_o)
    say(f"  {len(docs)} documents, R={R}, group {group}: Z within {worst:.3g} relative")
    return ll


@pytest.mark.parametrize("group", [16, 32, 64])
def test_heldout_matches_oracle_k100(group):
    c = synth.small_random(D=120, V=800, K=100, mean_len=220.0, seed=4)
    say(f"held-out K=100 group={group}")
    p = _model(c, seed=5)
    docs = _docs(c.V, [1, 2, 3, 7, 40, 130], seed=6)
    docs.append(np.array([c.V + 3, -1, 5, c.V, 9], np.int32))   # dropped ids among kept ones
    docs.append(np.zeros(0, np.int32))                             # empty
    _compare(p, c, docs, R=6, group=group, seed=11)


def test_heldout_k1000_and_dirichlet_phi():
    c = synth.small_random(D=50, V=3000, K=1000, mean_len=500.0, seed=5)
    say("held-out K=1000")
    for method in ("polya_urn", "dirichlet"):
        p = _model(c, seed=7, method=method)
        docs = _docs(c.V, [3, 60, 200], seed=8)
        _compare(p, c, docs, R=4, group=32, seed=12)


def test_heldout_deterministic_and_errors():
    c = synth.generate("tiny", keep_true_z=False)
    p = _model(c, seed=9)
    docs = _docs(c.V, [20, 35], seed=10)
    a = p.heldout_loglik(docs, particles=5, seed=3)
    b = p.heldout_loglik(docs, particles=5, seed=3)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    with pytest.raises(pulda.PuldaError):
        p.heldout_loglik(docs, particles=0)
    with pytest.raises(pulda.PuldaError):
        p.heldout_loglik(docs, group=8)
    with pytest.raises(pulda.PuldaError):
        p.heldout_loglik([np.zeros(70000, np.int32)], particles=1)
