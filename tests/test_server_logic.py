"""The continuous-batching loop, on the CPU, against a fake backend whose
requests are computed by the oracle's fold-in (no GPU)."""
import numpy as np
import pytest

import oracle
from paper_1704_03581_amd import server, synth


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeFoldIn:
    """FoldIn's interface with the oracle's arithmetic; one step (up to
    `draws` token draws per resident request) costs 1 ms of fake time."""

    def __init__(self, phi, wt, alpha, seed, clock, sweeps=8, burn_in=4, max_slots=4, arena_tokens=200):
        self.phi, self.wt, self.alpha, self.seed = phi, wt, alpha, seed
        self.clock = clock
        self.sweeps, self.burn_in = sweeps, burn_in
        self.max_slots, self.arena_tokens = max_slots, arena_tokens
        self.res = {}          # rid -> [words, draws done, step that finished it]
        self.used = 0
        self.submits = []
        self.steps = 0

    def submit(self, rid, words):
        if len(self.res) >= self.max_slots or self.used + max(len(words), 1) > self.arena_tokens:
            return False
        self.res[rid] = [np.asarray(words), 0, None]
        self.used += max(len(words), 1)
        self.submits.append(rid)
        return True

    def occupancy(self):
        return dict(resident=len(self.res), free_slots=self.max_slots - len(self.res),
                    free_tokens=self.arena_tokens - self.used)

    def step(self, draws):
        self.steps += 1
        for r in self.res.values():
            if r[2] is None:
                r[1] = min(self.sweeps * len(r[0]), r[1] + draws)
                if r[1] >= self.sweeps * len(r[0]):
                    r[2] = self.steps
        self.clock.t += 1e-3

    def _result(self, rid, words):
        theta, ll, kept, dropped, _ = oracle.foldin(self.phi, self.wt, self.alpha, self.seed, rid, words,
                                                    S=self.sweeps, burn_in=self.burn_in)
        return dict(request_id=rid, theta=theta, loglik=ll, kept=kept, dropped=dropped)

    def poll(self, cap=4096, previous=False):
        # previous: what the step before the latest finished (the latest runs on)
        limit = self.steps - 1 if previous else self.steps
        done = [rid for rid, r in self.res.items() if r[2] is not None and r[2] <= limit][:cap]
        out = []
        for rid in done:
            words, _, _ = self.res.pop(rid)
            self.used -= max(len(words), 1)
            out.append(self._result(rid, words))
        return out

    def run_one(self, rid, words):
        self.clock.t += 1e-3 * self.sweeps
        return self._result(rid, np.asarray(words))


@pytest.fixture(scope="module")
def model():
    c = synth.small_random(D=60, V=300, K=12, mean_len=40.0, seed=2)
    s = oracle.Sampler(c.doc_off, c.words, c.K, c.V, seed=4)
    for t in range(1, 4):
        s.sweep(t)
    return s.phi, s.wt, s.alpha


def _requests(n, V, seed):
    rng = np.random.default_rng(seed)
    return [rng.integers(0, V + 5, size=int(rng.integers(0, 60))).astype(np.int32) for _ in range(n)]


@pytest.mark.parametrize("pipelined", [True, False])
def test_all_served_fifo_and_identical_to_alone(model, pipelined):
    phi, wt, alpha = model
    reqs = _requests(30, phi.shape[1], 1)
    clk = FakeClock()
    be = FakeFoldIn(phi, wt, alpha, 9, clk)
    rep = server.serve(be, reqs, arrivals=None, draws=100, clock=clk, sleep=clk.sleep, pipelined=pipelined)
    assert sorted(rep.results) == list(range(30))
    assert rep.order_admitted == sorted(rep.order_admitted)          # first come, first served
    assert rep.max_resident <= be.max_slots and rep.admission_waits > 0
    for rid, r in rep.results.items():
        alone = be.run_one(rid, reqs[rid])
        assert np.array_equal(r["theta"], alone["theta"]) and r["loglik"] == alone["loglik"]
        assert r["kept"] + r["dropped"] == len(reqs[rid])


def test_admission_by_arena_tokens(model):
    """A request that does not fit waits (first come, first served: the small
    one behind it waits too) until a finished request frees arena space."""
    phi, wt, alpha = model
    reqs = [np.zeros(150, np.int32), np.zeros(150, np.int32), np.zeros(10, np.int32)]
    clk = FakeClock()
    be = FakeFoldIn(phi, wt, alpha, 9, clk, max_slots=8, arena_tokens=200)
    rep = server.serve(be, reqs, draws=8 * 150, clock=clk, sleep=clk.sleep)
    assert rep.admission_waits >= 1
    assert rep.order_admitted == [0, 1, 2]
    # 150 + 150 never fit together; 150 + 10 do
    assert rep.max_resident == 2


def test_request_larger_than_arena_is_an_error(model):
    phi, wt, alpha = model
    clk = FakeClock()
    be = FakeFoldIn(phi, wt, alpha, 9, clk, arena_tokens=50)
    with pytest.raises(RuntimeError):
        server.serve(be, [np.zeros(80, np.int32)], clock=clk, sleep=clk.sleep)


def test_open_loop_latency_arithmetic(model):
    """Latency = completion - arrival on the server's clock; percentiles from it."""
    phi, wt, alpha = model
    reqs = _requests(20, phi.shape[1], 3)
    arr = server.poisson_arrivals(20, rate=200.0, seed=5)
    clk = FakeClock()
    be = FakeFoldIn(phi, wt, alpha, 9, clk, max_slots=16, arena_tokens=10000)
    rep = server.serve(be, reqs, arrivals=arr, draws=60, clock=clk, sleep=clk.sleep)
    assert np.all(rep.latency_s > 0)
    # a request of n tokens needs ceil(8 n / 60) steps of 1 ms after admission
    need = np.array([max(1, -(-8 * len(r) // 60)) for r in reqs]) * 1e-3
    assert np.all(rep.latency_s >= need - 1e-12)
    assert rep.percentile_ms(50) <= rep.percentile_ms(99)
    assert abs(rep.percentile_ms(50) - np.percentile(rep.latency_s, 50) * 1e3) < 1e-9


def test_pipelined_collects_one_step_later(model):
    """The pipelined loop collects a request after the step following the
    one that finished it: the same results, each one step (1 ms) later, and
    the admissions that the freed slots allow shift by that step too."""
    phi, wt, alpha = model
    reqs = _requests(12, phi.shape[1], 6)
    reps = {}
    for pipelined in (False, True):
        clk = FakeClock()
        be = FakeFoldIn(phi, wt, alpha, 9, clk, max_slots=16, arena_tokens=10000)
        reps[pipelined] = server.serve(be, reqs, draws=100, clock=clk, sleep=clk.sleep, pipelined=pipelined)
    a, b = reps[False], reps[True]
    assert sorted(a.results) == sorted(b.results) == list(range(12))
    for rid in range(12):
        assert np.array_equal(a.results[rid]["theta"], b.results[rid]["theta"])
    # everything fits at once: each completion comes exactly one step later
    assert np.allclose(b.completion_s - a.completion_s, 1e-3)
    assert b.steps == a.steps + 1


def test_plain_sampler_same_results(model):
    phi, wt, alpha = model
    reqs = _requests(10, phi.shape[1], 4)
    clk = FakeClock()
    be = FakeFoldIn(phi, wt, alpha, 9, clk)
    rep_b = server.serve(be, reqs, draws=37, clock=clk, sleep=clk.sleep)
    rep_p = server.serve_plain(be, reqs, clock=clk, sleep=clk.sleep)
    for rid in range(10):
        assert np.array_equal(rep_b.results[rid]["theta"], rep_p.results[rid]["theta"])


def test_steady_rate_leaves_out_the_tail():
    """Completions at 1 per ms for 100 requests, then one straggler at 1 s:
    the steady rate is 1000/s, the plain rate is about 100/s."""
    comp = np.concatenate([np.arange(1, 101) * 1e-3, [1.0]])
    rep = server.ServeReport({i: {} for i in range(len(comp))}, comp.copy(), 1.0, completion_s=comp)
    assert abs(rep.steady_docs_per_s() - 1000.0) < 1e-6
    assert rep.docs_per_s < 110
