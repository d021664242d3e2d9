"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (autotuned schedule, all work-item classes), on outputs the
oracle can compute one by one.

* medium corpus (D=40000, K=1000, documents up to 20000 tokens): every
  token of one z-step replayed by the oracle, counts bit-exact;
* large corpus (D=8.2M, V=141000, K=1000, 738M tokens): the z-step of the
  fourth sweep after warmup and autotuning, as the benchmark runs it, with a
  sample of documents (random ones plus the longest and shortest) replayed
  by the oracle, the whole count table rebuilt by the z-step compared bit
  for bit, and the next Phi-step compared with the oracle's on every cell;
* fold-in against the large configuration's Phi (K=1000, V=141000), with the
  serving loop's draw budget: theta bit-exact and log-likelihood within
  1e-12 for requests of every length class;
* Algorithm 1's Dirichlet Phi-step on the large corpus's counts (141M
  cells): sampled Gamma draws against the oracle's per-cell draw, every row
  sum against an exact sum of the GPU's draws, phi within one fp32 ulp on the
  samples, and the z-step on that Phi replayed for sampled documents.

The large corpus is read from /tmp/pulda_large.npz when present (written by
`bench.py --generate-only`), otherwise generated (about a minute).
"""
import os

import numpy as np
import pytest

import oracle
from paper_1704_03581_amd import server, synth
from tests.gpu_helpers import assert_phi_equal, phi_from_gpu, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1704_03581_amd import pulda
else:
    pulda = None

LARGE_CACHE = "/tmp/pulda_large.npz"


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _plan(c, seed):
    p = pulda.Plan(c.K, c.V, c.D, c.N, alpha=c.alpha, beta=c.beta, seed=seed)
    p.upload(c.doc_off, c.words)
    p.init()
    return p


def _bench_like_zstep(p, t_warm):
    """Warmup sweeps, then autotuning on the state the timed sweeps start
    from, as the benchmark does; returns (z before, z after, Phi export) of
    the z-step of sweep t_warm + 1."""
    p.sweep(1, t_warm, want_ll=False)
    t = t_warm + 1
    p.phi_step(t)
    sched = p.autotune(t, reps=1)
    say(f"  schedule {sched}")
    z0 = p.get_z()
    p.phi_step(t)
    g = p.get_phi()
    p.z_step(t)
    return z0, p.get_z(), g, t


@pytest.mark.timeout(900)
def test_medium_every_token():
    _need_gpu()
    c = synth.generate("medium", keep_true_z=False)
    say(f"medium: D={c.D} N={c.N} longest={int(np.diff(c.doc_off).max())}")
    p = _plan(c, seed=31)
    z0, z1, g, t = _bench_like_zstep(p, 3)
    phi, wt = phi_from_gpu(g, c.K, c.V)
    r = oracle.replay(c.doc_off, c.words, z0, z1, 31, t, phi, wt, c.K, c.V)
    say(f"  replay {r}")
    assert r["bad"] == 0, r
    assert r["agree"] >= 0.9999 * c.N
    n_o, _, _ = oracle.counts(c.doc_off, c.words, z1, c.K, c.V, with_m=False)
    assert np.array_equal(p.counts_dense()[0], n_o)


@pytest.mark.timeout(900)
def test_large_sampled_documents():
    _need_gpu()
    if os.path.exists(LARGE_CACHE):
        c = synth.load(LARGE_CACHE)
    else:
        c = synth.generate("large", keep_true_z=False)
    say(f"large: D={c.D} N={c.N}")
    p = _plan(c, seed=1)
    z0, z1, g, t = _bench_like_zstep(p, 3)
    phi, wt = phi_from_gpu(g, c.K, c.V)
    del g
    lens = np.diff(c.doc_off)
    order = np.argsort(-lens, kind="stable")
    rng = np.random.default_rng(5)
    nonempty = order[lens[order] > 0]
    docs = np.unique(np.concatenate([rng.choice(c.D, 3000, replace=False), nonempty[:50], nonempty[-50:]]))
    n_tok = int(lens[docs].sum())
    r = oracle.replay(c.doc_off, c.words, z0, z1, 1, t, phi, wt, c.K, c.V, docs=docs)
    say(f"  replay of {len(docs)} documents ({n_tok} tokens): {r}")
    assert r["bad"] == 0, r
    assert r["agree"] >= 0.9999 * n_tok
    n_o, _, _ = oracle.counts(c.doc_off, c.words, z1, c.K, c.V, with_m=False)
    n_g, nk_g = p.counts_dense()
    assert np.array_equal(n_g, n_o)
    del n_o
    # the next sweep's Phi-step at full size, every cell against the
    # oracle's from the same counts: Poisson draws (alias tables, rounded
    # Gaussians above L, draws past the 16-bit range), prior marks, row sums,
    # phi, column layout, alias tables and sigma_a, bit for bit
    t2 = t + 1
    p.phi_step(t2)
    g = p.get_phi()
    gam = oracle.phi_counts(n_g, c.beta, 100, 1, t2)
    S, phi2, _ = oracle.phi_normalise(gam)
    wt2 = oracle.word_tables(np.full(c.K, c.alpha), phi2)
    say(f"  Phi-step t={t2}: nnz {len(wt2.topic)}, counted cells {int((n_g > 0).sum())}, "
        f"cells with n > 100 {int((n_g > 100).sum())}, draws >= 0xFFFF {int((gam >= 0xFFFF).sum())}, "
        f"largest column {int(np.diff(wt2.colptr).max())}, largest S_k {int(S.max())}")
    assert_phi_equal(g, gam, S, phi2, wt2, c.K, c.V)


@pytest.mark.timeout(600)
def test_foldin_large_model():
    _need_gpu()
    cfg = synth.CONFIGS["large"]
    K, V = cfg["K"], cfg["V"]
    n = synth.topic_word_counts_draw("large")
    model = pulda.Plan(K, V, 0, 0, alpha=synth.ALPHA, beta=synth.BETA, seed=7)
    model.set_counts(np.ascontiguousarray(n.T).reshape(-1))
    del n
    model.phi_step(1)
    phi, wt = phi_from_gpu(model.get_phi(), K, V)
    reqs = synth.foldin_requests(400, seed=11)
    lens = np.array([len(r) for r in reqs])
    order = np.argsort(lens)
    pick = np.unique(np.concatenate([order[:4], order[len(order) // 2 - 4:len(order) // 2 + 4], order[-4:]]))
    sub = [reqs[i] for i in pick]
    say(f"fold-in, lengths {sorted(len(r) for r in sub)}")
    f = pulda.FoldIn(model, sweeps=50, burn_in=25, max_slots=8, arena_tokens=20000, max_len=5000, group=64,
                     seed=13)
    rep = server.serve(f, sub, draws=2048)
    alpha = np.full(K, synth.ALPHA)
    for rid, res in rep.results.items():
        theta, ll, kept, dropped, _ = oracle.foldin(phi, wt, alpha, 13, rid, sub[rid], S=50, burn_in=25)
        assert res["kept"] == kept and res["dropped"] == dropped
        assert np.array_equal(res["theta"], theta), rid
        assert abs(res["loglik"] - ll) <= 1e-12 * abs(ll), (rid, res["loglik"], ll)


@pytest.mark.timeout(900)
def test_large_dirichlet_phi_and_z_step():
    import math
    _need_gpu()
    if os.path.exists(LARGE_CACHE):
        c = synth.load(LARGE_CACHE)
    else:
        c = synth.generate("large", keep_true_z=False)
    say(f"large, Dirichlet Phi: D={c.D} N={c.N}")
    p = _plan(c, seed=3)
    p.sweep(1, 2, want_ll=False)
    p.set_phi_method("dirichlet")
    t = 3
    n, _ = p.counts_dense()
    z0 = p.get_z()
    p.phi_step(t)
    gam, S = p.gamma_dense()
    rng = np.random.default_rng(9)
    ks = rng.integers(0, c.K, 4000)
    vs = rng.integers(0, c.V, 4000)
    # counted cells too: the most frequent word's column
    top = int(np.argmax(n.sum(axis=0)))
    ks = np.concatenate([ks, np.arange(c.K)])
    vs = np.concatenate([vs, np.full(c.K, top)])
    g_o = np.array([oracle.gamma_draw(c.beta + float(n[k, v]), 3, int(v), int(k), t) for k, v in zip(ks, vs)])
    g_g = gam[ks, vs]
    scale = np.maximum(np.abs(g_g), np.abs(g_o))
    rel = np.abs(g_g - g_o) / np.where(scale > 0, scale, 1.0)
    say(f"  {len(ks)} sampled Gamma draws: max relative difference {rel.max():.3g}")
    assert np.all(np.abs(g_g - g_o) <= 1e-12 * scale + 1e-300)
    # every row against numpy's sum, 50 rows against an exactly rounded sum
    assert np.all(np.abs(S - gam.sum(axis=1)) <= 2 * c.V * 2.0 ** -52 * S)
    for k in rng.choice(c.K, 50, replace=False):
        exact = math.fsum(gam[k])
        assert abs(S[k] - exact) <= c.V * 2.0 ** -52 * exact
    g = p.get_phi()
    phi, wt = phi_from_gpu(g, c.K, c.V)
    del g
    q = (g_g / S[ks]).astype(np.float32)
    q = np.where(q >= np.finfo(np.float32).tiny, q, 0).astype(np.float32)
    d = np.abs(phi[ks, vs].view(np.int32).astype(np.int64) - q.view(np.int32).astype(np.int64))
    assert d.max() <= 1
    del gam
    p.z_step(t)
    z1 = p.get_z()
    lens = np.diff(c.doc_off)
    docs = np.unique(rng.choice(np.nonzero(lens)[0], 2000, replace=False))
    r = oracle.replay(c.doc_off, c.words, z0, z1, 3, t, phi, wt, c.K, c.V, docs=docs)
    n_tok = int(lens[docs].sum())
    say(f"  replay of {len(docs)} documents ({n_tok} tokens): {r}")
    assert r["bad"] == 0, r
    assert r["agree"] >= 0.9999 * n_tok
