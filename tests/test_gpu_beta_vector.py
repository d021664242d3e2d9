"""GPU parity with per-word priors beta_v (the paper's beta is a V-vector),
through the C ABI, against the CPU oracle: the Polya-urn Phi-step bit for bit
(integer draws, tables and thresholds built on the host like the oracle's),
the log joint within 1e-10 (lgamma from the device library), the z-step by
replay, and the Dirichlet Phi-step's Gamma draws within 1e-12."""
import numpy as np
import pytest

import oracle
from paper_1704_03581_amd import synth
from tests.gpu_helpers import assert_phi_equal, oracle_phi, phi_from_gpu, say

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


CASES = {
    "k100": lambda: synth.small_random(D=120, V=800, K=100, mean_len=220.0, seed=4),
    "k1000": lambda: synth.small_random(D=50, V=3000, K=1000, mean_len=500.0, seed=5),
}


def _beta_v(V, seed):
    rng = np.random.default_rng(seed)
    # mostly small priors, a few large ones (multi-entry zero-truncated tables)
    b = rng.uniform(0.002, 0.05, V)
    b[rng.choice(V, V // 20, replace=False)] = rng.uniform(0.5, 6.0, V // 20)
    return b


@pytest.mark.parametrize("name", list(CASES))
def test_beta_vector_phi_loglik_and_z(name):
    c = CASES[name]()
    bv = _beta_v(c.V, 3)
    say(f"beta_v {name}")
    p = pulda.Plan(c.K, c.V, c.D, c.N, alpha=c.alpha, beta=bv, seed=15)
    p.upload(c.doc_off, c.words)
    p.init()
    for t in (1, 2):
        z0 = p.get_z()
        p.phi_step(t)
        g = p.get_phi()
        gam, S, phi, wt = oracle_phi(c.doc_off, c.words, z0, c.K, c.V, c.alpha, 0.01, 100, 15, t, beta_v=bv)
        assert_phi_equal(g, gam, S, phi, wt, c.K, c.V)
        phi_g, wt_g = phi_from_gpu(g, c.K, c.V)
        p.z_step(t)
        z1 = p.get_z()
        r = oracle.replay(c.doc_off, c.words, z0, z1, 15, t, phi_g, wt_g, c.K, c.V)
        say(f"  t={t} replay {r}")
        assert r["bad"] == 0, r
        ll_o = oracle.loglik(c.doc_off, c.words, z1, c.alpha, 0.01, c.K, c.V, beta_v=bv)
        assert abs(p.loglik() - ll_o) <= 1e-10 * abs(ll_o)


def test_beta_vector_sweeps_and_dirichlet():
    c = CASES["k100"]()
    bv = _beta_v(c.V, 4)
    p = pulda.Plan(c.K, c.V, c.D, c.N, alpha=c.alpha, beta=bv, seed=17)
    p.upload(c.doc_off, c.words)
    p.init()
    lls = p.sweep(1, 3)
    ll_o = oracle.loglik(c.doc_off, c.words, p.get_z(), c.alpha, 0.01, c.K, c.V, beta_v=bv)
    assert abs(lls[-1] - ll_o) <= 1e-10 * abs(ll_o)
    p.set_phi_method("dirichlet")
    n, _ = p.counts_dense()
    p.phi_step(4)
    gam_g, S_g = p.gamma_dense()
    gam_o, S_o, _, _ = oracle.phi_dirichlet(n, 0.01, 17, 4, beta_v=bv)
    scale = np.maximum(np.abs(gam_g), np.abs(gam_o))
    assert np.all(np.abs(gam_g - gam_o) <= 1e-12 * scale + 1e-300)
    assert np.all(np.abs(S_g - S_o) <= c.V * 2.0 ** -52 * S_o * 1.01)
