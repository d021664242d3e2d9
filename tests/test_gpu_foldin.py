"""Fold-in on the GPU (through the C ABI) against the oracle's fold-in.

theta is computed from integer topic counts, so it must match bit for bit
whenever the draws match; the draws use the same fp64 token law as the
z-step, so they are compared exactly too (a floating-point tie would show as
a mismatch here and has probability ~1e-13 per draw).  The log-likelihood
of the final state is a sum in a different order: 1e-12 relative.
"""
import numpy as np
import pytest

import oracle
from paper_1704_03581_amd import server, synth
from tests.gpu_helpers import phi_from_gpu, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1704_03581_amd import pulda
else:
    pulda = None


@pytest.fixture(scope="module")
def model():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = synth.small_random(D=200, V=2000, K=64, mean_len=80.0, seed=12)
    p = pulda.Plan(c.K, c.V, c.D, c.N, alpha=c.alpha, beta=c.beta, seed=3)
    p.upload(c.doc_off, c.words)
    p.init()
    p.sweep(1, 5, want_ll=False)
    p.phi_step(6)
    phi, wt = phi_from_gpu(p.get_phi(), c.K, c.V)
    return p, phi, wt, c


def _requests(V, n, seed):
    rng = np.random.default_rng(seed)
    reqs = [rng.integers(0, V, size=int(rng.integers(10, 300))).astype(np.int32) for _ in range(n)]
    reqs.append(np.zeros(0, np.int32))                                  # empty request
    reqs.append(np.array([V, V + 7, -1], np.int32))                     # all out of range
    reqs.append(np.concatenate([reqs[0][:20], [V + 1, V + 2]]).astype(np.int32))
    return reqs


def _check(res, phi, wt, alpha, seed, rid, words, sweeps, burn_in):
    theta, ll, kept, dropped, _ = oracle.foldin(phi, wt, alpha, seed, rid, words, S=sweeps, burn_in=burn_in)
    assert res["kept"] == kept and res["dropped"] == dropped, (rid, res["kept"], kept)
    assert np.array_equal(res["theta"], theta), rid
    assert abs(res["loglik"] - ll) <= 1e-12 * max(1.0, abs(ll)), (rid, res["loglik"], ll)


@pytest.mark.parametrize("group", [64, 32, 16])
def test_foldin_batched_matches_oracle(model, group):
    p, phi, wt, c = model
    say(f"fold-in batched group={group}")
    f = pulda.FoldIn(p, sweeps=12, burn_in=6, max_slots=16, arena_tokens=4000, max_len=400, group=group, seed=21)
    reqs = _requests(c.V, 40, 5)
    rep = server.serve(f, reqs, draws=300)
    assert sorted(rep.results) == list(range(len(reqs)))
    for rid, r in rep.results.items():
        _check(r, phi, wt, np.full(c.K, c.alpha), 21, rid, reqs[rid], 12, 6)


def test_foldin_alone_equals_in_the_mix(model):
    """Each request's result is the same alone (plain sampler) and among
    others with any budget of draws per step (steps that stop mid-sweep
    included)."""
    p, phi, wt, c = model
    say("fold-in alone vs mix")
    f = pulda.FoldIn(p, sweeps=10, burn_in=5, max_slots=8, arena_tokens=2000, max_len=400, group=64, seed=33)
    reqs = _requests(c.V, 20, 8)
    alone = {rid: f.run_one(rid, w) for rid, w in enumerate(reqs)}
    # both serving loops: collecting each step's results after it (the poll
    # waits for the step) and the previous step's while the next one runs
    for q, pipelined in ((7, True), (100, True), (1000, True), (100, False)):
        rep = server.serve(f, reqs, draws=q, pipelined=pipelined)
        assert sorted(rep.results) == list(range(len(reqs)))
        for rid, r in rep.results.items():
            assert np.array_equal(r["theta"], alone[rid]["theta"]) and r["loglik"] == alone[rid]["loglik"]
    _check(alone[0], phi, wt, np.full(c.K, c.alpha), 33, 0, reqs[0], 10, 5)


def test_foldin_admission_under_memory_cap(model):
    """A small arena admits few requests at once; the rest wait, none fail."""
    p, phi, wt, c = model
    say("fold-in admission")
    f = pulda.FoldIn(p, sweeps=6, burn_in=3, max_slots=32, arena_tokens=500, max_len=300, group=32, seed=5)
    reqs = _requests(c.V, 25, 9)
    with pytest.raises(pulda.PuldaError):
        f.submit(999, np.zeros(301, np.int32))                          # longer than max_len
    rep = server.serve(f, reqs, draws=150)
    assert rep.admission_waits > 0 and sorted(rep.results) == list(range(len(reqs)))
    occ = f.occupancy()
    assert occ["resident"] == 0 and occ["free_tokens"] == 500 and occ["free_slots"] == 32
    for rid in (0, 5, 24):
        _check(rep.results[rid], phi, wt, np.full(c.K, c.alpha), 5, rid, reqs[rid], 6, 3)


def test_foldin_poll_previous_lags_one_step(model):
    """pulda_foldin_poll_previous reports what the step before the latest
    finished: nothing after the first step, a request finished by step s
    after step s+1 (whose launch skips it), the same results as the
    synchronous poll."""
    p, phi, wt, c = model
    say("fold-in lagged poll")
    reqs = _requests(c.V, 6, 11)[:6]
    f = pulda.FoldIn(p, sweeps=4, burn_in=2, max_slots=8, arena_tokens=4000, max_len=400, group=64, seed=17)
    alone = {rid: f.run_one(rid, w) for rid, w in enumerate(reqs)}
    for rid, w in enumerate(reqs):
        assert f.submit(rid, w)
    big = 1 << 30
    f.step(big)                                   # every request finishes in this step
    assert f.poll(previous=True) == []            # nothing before the second step
    f.step(big)                                   # finished ones are skipped
    got = {r["request_id"]: r for r in f.poll(previous=True)}
    assert sorted(got) == list(range(len(reqs)))
    for rid, r in got.items():
        assert np.array_equal(r["theta"], alone[rid]["theta"]) and r["loglik"] == alone[rid]["loglik"]
    assert f.occupancy()["resident"] == 0
