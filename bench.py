"""Benchmark: z-step tokens/s at K=1000 and fold-in serving, on one MI355X.

One step = one sweep of Algorithm 2 over the whole synthetic corpus:
Phi-step (Poisson Polya urn draws, per-word alias tables), z-step with the
count rebuild, and the collapsed log joint.  Inputs are resident in HBM
before the timed region.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--config large]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, AMD's published figure


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(N, sum_J, sum_A):
    """Bytes the doubly sparse z-step must touch per sweep (per token:
    word id 4, z read 2 and write 2, the column's two offsets 8, sigma_a 4,
    the count increment 8, plus 6 per b-term (u16 topic + fp32 phi) and 8
    per a-part alias bucket)."""
    return 28 * N + 6 * sum_J + 8 * sum_A


def kernel_source_hash():
    """sha256 prefix of the z-step kernel sources; a recorded counter reading
    applies only to the kernel it was taken on."""
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels.hip", "device.h"):
        with open(os.path.join(ROOT, "paper_1704_03581_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(config):
    """HBM bytes per z-step launch from the committed FETCH_SIZE/WRITE_SIZE
    counter summary (already scaled by the 1 GiB copy calibration), or None
    when the summary is for another workload or an older kernel."""
    path = os.path.join(ROOT, "profiles", f"zstep_{config}_counters.txt")
    if not os.path.exists(path):
        return None, None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.strip().split("=", 1)
                kv[k] = v
    if kv.get("kernel_source_hash") != kernel_source_hash():
        return None, path
    return float(kv["traffic_bytes_per_launch"]), path


def host_cpu():
    """The host's CPU model (lscpu's model name) and its core count."""
    model = "unknown"
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    return model, os.cpu_count()


def cpu_baseline(corpus, seed, budget_docs):
    """The oracle (single-threaded C) on a bounded sample of the same corpus:
    its doubly sparse z-step mode (bit-identical to its dense definition),
    pinned to one core, one sweep from the initial state."""
    import oracle
    d = min(budget_docs, corpus.D)
    off = corpus.doc_off[: d + 1].copy()
    words = corpus.words[: off[-1]].copy()
    n_tok = int(off[-1])
    z = oracle.init_z(n_tok, corpus.K, seed)
    alpha = np.full(corpus.K, corpus.alpha)
    model, ncpu = host_cpu()
    old_aff = os.sched_getaffinity(0) if hasattr(os, "sched_getaffinity") else None
    if old_aff:
        os.sched_setaffinity(0, {min(old_aff)})
    try:
        t0 = time.perf_counter()
        n, _, _ = oracle.counts(off, words, z, corpus.K, corpus.V, with_m=False)
        gam = oracle.phi_counts(n, corpus.beta, 100, seed, 1)
        S, phi, _ = oracle.phi_normalise(gam)
        wt = oracle.word_tables(alpha, phi)
        t1 = time.perf_counter()
        oracle.z_step(off, words, z, seed, 1, phi, wt, corpus.K, corpus.V, sparse=True)
        t2 = time.perf_counter()
        oracle.loglik(off, words, z, alpha, corpus.beta, corpus.K, corpus.V)
        t3 = time.perf_counter()
    finally:
        if old_aff:
            os.sched_setaffinity(0, old_aff)
    return dict(value=n_tok / (t2 - t1), unit="tokens/s", cores=1, kind="oracle",
                sample=f"first {d} documents ({n_tok} tokens) of the same corpus, one sweep from the "
                       f"initial state, the oracle's doubly sparse z-step (bit-identical to its dense mode) on one "
                       f"pinned core; z-step {t2 - t1:.2f}s, Phi-step {t1 - t0:.2f}s, log joint {t3 - t2:.2f}s",
                host_cpu=model, host_cores=ncpu, sweep_tokens_per_s=n_tok / (t3 - t0))


def foldin_bench(args, torch, pulda, synth, model=None, phi_source=None):
    """Fold-in serving against a resident Phi (K=1000, V=141000): continuous
    batching (closed loop, then open-loop Poisson arrivals of at least
    args.trace_s seconds per rate) and the plain per-document sampler on the
    same requests.  model: a plan holding the serving Phi (default: a Phi-step
    from counts drawn from the generating topics, see phi_source)."""
    from paper_1704_03581_amd import server
    cfg = synth.CONFIGS["large"]
    K, V = cfg["K"], cfg["V"]
    if model is None:
        log("fold-in: drawing serving counts and Phi")
        n = synth.topic_word_counts_draw("large")
        model = pulda.Plan(K, V, 0, 0, alpha=synth.ALPHA, beta=synth.BETA, seed=args.seed)
        model.set_counts(np.ascontiguousarray(n.T).reshape(-1))
        del n
        model.phi_step(1)
        phi_source = ("one Phi-step from topic-word counts drawn from the generating topics (738M tokens); "
                      "bench.py --converged serves the Phi of a 1000-sweep run")
    torch.cuda.synchronize()
    # enough requests for trace_s seconds of arrivals at the highest rate
    n_trace = args.foldin_requests
    reqs = synth.foldin_requests(max(n_trace, 1) + max(args.plain_requests, args.foldin_cpu_requests),
                                 seed=170403581 + 5)
    lens = np.array([len(r) for r in reqs])
    fi = pulda.FoldIn(model, sweeps=50, burn_in=25, max_slots=args.slots, arena_tokens=args.slots * 600,
                      max_len=5000, group=args.foldin_group, seed=args.seed)
    nb = min(args.closed_requests, n_trace)
    batched = reqs[:nb]
    log(f"fold-in: closed loop, {nb} requests")
    rep = server.serve(fi, batched, draws=args.draws)
    # the service rate: completions between the 10% and 90% marks (the run's
    # end waits for its longest requests, 50 sweeps of up to 5000 tokens)
    xmax = rep.steady_docs_per_s()
    out = dict(phi=phi_source, service_rate_docs_per_s=xmax, closed_loop_docs_per_s=rep.docs_per_s,
               closed_loop_p50_ms=rep.percentile_ms(50), closed_loop_p99_ms=rep.percentile_ms(99),
               closed_loop_requests=nb, mean_len=float(lens[:n_trace].mean()),
               closed_loop_steps=rep.steps, closed_loop_ms_per_step=1e3 * rep.wall_s / max(rep.steps, 1),
               sweeps=50, burn_in=25, slots=args.slots, draws_per_step=args.draws, group=args.foldin_group,
               trace_s=args.trace_s,
               rates={})
    sustained = 0.0
    for i, frac in enumerate(args.rates):
        # open loop: Poisson arrivals for trace_s seconds at frac x the
        # service rate; delivered rate and latencies over the arrivals
        # between the 10% and 90% marks (start-up and drain left out)
        rate = frac * xmax
        n_req = min(n_trace, max(1000, int(rate * args.trace_s)))
        arr = server.poisson_arrivals(n_req, rate, seed=170403581 + 5 + i)
        rep = server.serve(fi, reqs[:n_req], arrivals=arr, draws=args.draws)
        delivered, p50, p99 = rep.arrival_window(arr)
        out["rates"][f"{frac:.2f}"] = dict(offered_docs_per_s=rate, requests=n_req, arrival_s=float(arr[-1]),
                                           delivered_docs_per_s=delivered, p50_ms=p50, p99_ms=p99,
                                           whole_run_docs_per_s=rep.docs_per_s, max_resident=rep.max_resident,
                                           steps=rep.steps, ms_per_step=1e3 * rep.wall_s / max(rep.steps, 1))
        if delivered >= 0.97 * rate:
            sustained = max(sustained, rate)
        log(f"fold-in: rate {frac:.2f} x -> {out['rates'][f'{frac:.2f}']}")
    out["sustained_docs_per_s"] = sustained
    plain = reqs[n_trace:n_trace + args.plain_requests]
    rep_p = server.serve_plain(fi, plain)
    out["plain_docs_per_s"] = rep_p.docs_per_s
    out["plain_p50_ms"] = rep_p.percentile_ms(50)
    out["plain_p99_ms"] = rep_p.percentile_ms(99)
    # the same requests through the batched path give the same results
    rep_b = server.serve(fi, plain, draws=args.draws)
    out["batched_equals_plain"] = bool(all(
        np.array_equal(rep_b.results[j]["theta"], rep_p.results[j]["theta"]) and
        rep_b.results[j]["loglik"] == rep_p.results[j]["loglik"] for j in range(len(plain))))
    # like with like: whole-run rate against whole-run rate (the closed loop
    # includes its start-up and its drain; the plain sampler, one request at
    # a time, has neither, so its rate does not depend on the count)
    out["speedup_vs_plain"] = out["closed_loop_docs_per_s"] / out["plain_docs_per_s"]
    # and the steady service rate against the same plain rate
    out["service_rate_vs_plain"] = xmax / out["plain_docs_per_s"]
    if args.foldin_cpu_requests > 0 and not args.no_cpu_baseline:
        # the oracle's fold-in (single-threaded, one pinned core) on the
        # requests the plain sampler takes (and more after them), same Phi,
        # request ids and seed; its theta must equal the GPU's bit for bit
        import oracle
        phi, wt = oracle_tables(model, K, V)
        a = np.full(K, synth.ALPHA)
        sub = reqs[n_trace:n_trace + args.foldin_cpu_requests]
        old_aff = os.sched_getaffinity(0) if hasattr(os, "sched_getaffinity") else None
        try:
            if old_aff:
                os.sched_setaffinity(0, {min(old_aff)})
            t0 = time.perf_counter()
            same = True
            for j, wj in enumerate(sub):
                theta, ll, kept, _, _ = oracle.foldin(phi, wt, a, args.seed, j, wj, S=50, burn_in=25)
                if j in rep_p.results:
                    same &= bool(np.array_equal(theta, rep_p.results[j]["theta"]) and kept == rep_p.results[j]["kept"])
            dto = time.perf_counter() - t0
        finally:
            if old_aff:
                os.sched_setaffinity(0, old_aff)
        draws = 50 * sum(len(w) for w in sub)
        out["cpu_baseline"] = dict(kind="oracle", cores=1, requests=len(sub), docs_per_s=len(sub) / dto,
                                   token_draws_per_s=draws / dto, seconds=dto,
                                   theta_equal_gpu=same, compared=min(len(sub), len(plain)))
    return out


def oracle_tables(plan, K, V):
    """The plan's current Phi as the oracle takes it: dense fp32 phi (K x V)
    and the per-word tables (CSC, alias tables, sigma_a), read back from the
    GPU."""
    import oracle
    g = plan.get_phi()
    colptr = g["colptr"].astype(np.int64)
    cols = np.repeat(np.arange(V), np.diff(colptr))
    phi = np.zeros((K, V), np.float32)
    phi[g["topic"].astype(np.int64), cols] = g["phi"]
    wt = oracle.WordTables(colptr, g["topic"].astype(np.uint16), g["phi"].astype(np.float32),
                           g["alias_thr"].astype(np.uint32), g["alias_topic"].astype(np.uint16),
                           g["sigma_a"].astype(np.float64))
    return phi, wt


def heldout_bench(plan, docs, particles, seed, torch, oracle_docs=0, K=0, V=0, alpha=0.0):
    """Held-out log-likelihood of new documents (left-to-right estimate, as in
    the paper's Section 4) against the plan's current Phi: wall time of the
    call (document upload included), token draws per second, and the
    estimate per token; optionally the oracle on the first few documents."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ll, kept = plan.heldout_loglik(docs, particles=particles, group=32, seed=seed)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n = kept.astype(np.int64)
    draws = int(particles * (n * (n + 1) // 2).sum())
    out = dict(docs=len(docs), particles=particles, tokens=int(n.sum()), max_len=int(n.max()), seconds=dt,
               docs_per_s=len(docs) / dt, token_draws_per_s=draws / dt, ll_per_token=float(ll.sum() / n.sum()))
    if oracle_docs:
        # the oracle (single-threaded) on the first few documents, same Phi
        import oracle
        phi, wt = oracle_tables(plan, K, V)
        a = np.full(K, alpha)
        sub = docs[:oracle_docs]
        t0 = time.perf_counter()
        nd = 0
        for i, d in enumerate(sub):
            _, k = oracle.heldout_ltr(phi, wt, a, seed, i, d, particles)
            nd += particles * k * (k + 1) // 2
        dto = time.perf_counter() - t0
        out["cpu_baseline"] = dict(kind="oracle", cores=1, docs=len(sub), docs_per_s=len(sub) / dto,
                                   token_draws_per_s=nd / dto, seconds=dto)
    return out


def scaling_study(args, torch, pulda, synth):
    """Where the urn's speedup comes from (the paper's Section 4 scaling
    study): both Phi-steps with the same z-step on restrictions of the large
    corpus by rare-word limit, vocabulary size and data size.  Per
    configuration: 3 warmup sweeps with the urn, 5 timed urn sweeps, then 5
    timed sweeps with the Dirichlet Phi-step continuing the chain; per-phase
    hipEvent times.  (The large corpus fills the GPU with short documents; on
    a smaller one each z-step waits for its longest document's chain.)"""
    if args.corpus_cache and os.path.exists(args.corpus_cache):
        base = synth.load(args.corpus_cache)
    else:
        base = synth.generate("large", keep_true_z=False)
    grid = ([dict(min_count=m) for m in (0, 10, 50, 200)] +
            [dict(max_vocab=v) for v in (2000, 5000, 10000)] +
            [dict(doc_fraction=f) for f in (0.125, 0.25, 0.5)])
    rows = []
    for g in grid:
        c = synth.restrict(base, **g)
        plan = pulda.Plan(c.K, c.V, c.D, c.N, alpha=c.alpha, beta=c.beta, seed=args.seed)
        plan.upload(c.doc_off, c.words)
        plan.init()
        plan.sweep(1, 3, want_ll=False)
        plan.set_timing(True)
        row = dict(g, V=c.V, N=c.N)
        for method, t0 in (("polya_urn", 4), ("dirichlet", 9)):
            plan.set_phi_method(method)
            plan.stats()
            plan.sweep(t0, 5, want_ll=False)
            st = plan.stats()
            row[method] = dict(phi_ms=st["ms_phi"] / st["n_phi"], z_ms=st["ms_z"] / st["n_z"], nnz_phi=st["nnz_phi"],
                               mean_J=st["sum_J"] / st["z_steps"] / c.N)
        row["z_ratio"] = row["dirichlet"]["z_ms"] / row["polya_urn"]["z_ms"]
        row["phi_ratio"] = row["dirichlet"]["phi_ms"] / row["polya_urn"]["phi_ms"]
        log(f"scaling {row}")
        rows.append(row)
        del plan
        torch.cuda.empty_cache()
    return dict(workload=f"large corpus (D={base.D}, V={base.V}, K={base.K}, N={base.N}) restricted by rare-word "
                         f"limit, vocabulary size and data size", rows=rows)


def ksweep_study(args, torch, pulda, synth):
    """The paper's K comparison (Section 4: K = 10, 100, 1000; time per
    iteration of both samplers and their log-posterior traces) on synthetic
    data: both Phi-steps with the same z-step at each K on the large corpus
    (3 warmup sweeps, autotuned schedule, 5 timed sweeps of each method
    continuing the chain, per-phase hipEvent times), and per-sweep log-joint
    traces of Algorithm 2 and Algorithm 1 from the same initial state on an
    eighth of its documents (args.trace_sweeps sweeps each)."""
    if args.corpus_cache and os.path.exists(args.corpus_cache):
        base = synth.load(args.corpus_cache)
    else:
        base = synth.generate("large", keep_true_z=False)
    small = synth.restrict(base, doc_fraction=0.125)
    rows = []
    for K in args.ks:
        plan = pulda.Plan(K, base.V, base.D, base.N, alpha=base.alpha, beta=base.beta, seed=args.seed)
        plan.upload(base.doc_off, base.words)
        plan.init()
        plan.sweep(1, 3, want_ll=False)
        plan.phi_step(4)
        sched = plan.autotune(4, reps=1)
        plan.set_timing(True)
        row = dict(K=K, N=base.N, schedule=sched)
        for method, t0 in (("polya_urn", 4), ("dirichlet", 9)):
            plan.set_phi_method(method)
            plan.stats()
            plan.sweep(t0, 5, want_ll=False)
            st = plan.stats()
            z_ms = st["ms_z"] / st["n_z"]
            row[method] = dict(phi_ms=st["ms_phi"] / st["n_phi"], z_ms=z_ms, ll_ms=st["ms_ll"] / max(st["n_ll"], 1),
                               z_tokens_per_s=base.N / (z_ms * 1e-3), nnz_phi=st["nnz_phi"],
                               mean_J=st["sum_J"] / st["z_steps"] / base.N,
                               a_fraction=st["sum_A"] / st["z_steps"] / base.N)
        row["z_ratio_dirichlet_over_urn"] = row["dirichlet"]["z_ms"] / row["polya_urn"]["z_ms"]
        row["phi_ratio_dirichlet_over_urn"] = row["dirichlet"]["phi_ms"] / row["polya_urn"]["phi_ms"]
        del plan
        torch.cuda.empty_cache()
        # log-joint traces of both samplers from the same initial state
        traces = {}
        for method in ("polya_urn", "dirichlet"):
            tp = pulda.Plan(K, small.V, small.D, small.N, alpha=small.alpha, beta=small.beta, seed=args.seed)
            tp.upload(small.doc_off, small.words)
            tp.init()
            tp.set_phi_method(method)
            lls = []
            for t in range(1, args.trace_sweeps + 1, 50):
                n = min(50, args.trace_sweeps + 1 - t)
                lls.extend(tp.sweep(t, n))
            traces[method] = np.asarray(lls)
            del tp
            torch.cuda.empty_cache()
        marks = [1, 2, 5, 10, 20, 50, 100, 200, 300, 500, 1000]
        marks = [m for m in marks if m <= args.trace_sweeps]
        row["trace"] = dict(corpus=f"an eighth of the documents (D={small.D}, N={small.N})",
                            sweeps=marks,
                            polya_urn=[float(traces["polya_urn"][m - 1]) for m in marks],
                            dirichlet=[float(traces["dirichlet"][m - 1]) for m in marks])
        tail = max(1, args.trace_sweeps // 4)
        u, d = traces["polya_urn"][-tail:], traces["dirichlet"][-tail:]
        row["trace"]["last_quarter_mean"] = dict(polya_urn=float(u.mean()), dirichlet=float(d.mean()),
                                                 relative_gap=float((u.mean() - d.mean()) / abs(d.mean())),
                                                 polya_urn_sd=float(u.std()), dirichlet_sd=float(d.std()))
        log(f"ksweep K={K}: {json.dumps({k: v for k, v in row.items() if k != 'trace'})}")
        log(f"ksweep K={K} trace: {json.dumps(row['trace'])}")
        rows.append(row)
    return dict(workload=f"large corpus (D={base.D}, V={base.V}, N={base.N}, generated with K=1000) sampled with "
                         f"K = 10, 100, 1000", rows=rows)


def converged_study(args, torch, pulda, synth):
    """The large workload run for 1000 sweeps: z-step throughput over the
    first sweeps (dense initial state) and over sweeps 901-1000 (converged),
    both with per-phase events and a schedule autotuned on that state, the
    sweeps between replayed from a captured graph; log joint every 100
    sweeps; then fold-in serving against the Phi of sweep 1001, as the
    serving workload specifies."""
    if args.corpus_cache and os.path.exists(args.corpus_cache):
        c = synth.load(args.corpus_cache)
    else:
        c = synth.generate("large", keep_true_z=False)
    N = c.N
    plan = pulda.Plan(c.K, c.V, c.D, c.N, alpha=c.alpha, beta=c.beta, seed=args.seed)
    plan.upload(c.doc_off, c.words)
    plan.init()

    def window(t0, n):
        plan.set_graph(False)
        plan.phi_step(t0)
        sched = plan.autotune(t0, reps=1)
        plan.set_timing(True)
        plan.stats()
        plan.sweep(t0, n, want_ll=False)
        st = plan.stats()
        plan.set_timing(False)
        z_ms = st["ms_z"] / st["n_z"]
        bytes_launch = algorithmic_bytes(N, st["sum_J"] / st["z_steps"], st["sum_A"] / st["z_steps"])
        bytes_b = algorithmic_bytes(N, st["sum_J_b"] / st["z_steps"], st["sum_A"] / st["z_steps"])
        return dict(sweeps=[t0, t0 + n - 1], schedule=sched, z_ms=z_ms, z_tokens_per_s=N / (z_ms * 1e-3),
                    phi_ms=st["ms_phi"] / st["n_phi"], loglik_ms=st["ms_ll"] / max(st["n_ll"], 1),
                    sweep_ms=(st["ms_phi"] + st["ms_z"] + st["ms_ll"]) / st["n_z"],
                    mean_J=st["sum_J"] / st["z_steps"] / N, mean_J_b_terms_read=st["sum_J_b"] / st["z_steps"] / N,
                    a_fraction=st["sum_A"] / st["z_steps"] / N, nnz_phi=st["nnz_phi"],
                    frac=bytes_launch / (z_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    frac_b_terms_read=bytes_b / (z_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, loglik=plan.loglik())

    out = dict(workload=f"large: D={c.D} V={c.V} K={c.K} N={N}", lls={})
    log("converged: sweeps 1-10")
    out["first"] = window(1, 10)
    log(f"converged: first window {out['first']}")
    plan.set_graph(True)
    t = 11
    w0 = time.perf_counter()
    for target in range(101, 902, 100):
        plan.sweep(t, target - t, want_ll=False)
        t = target
        out["lls"][t - 1] = plan.loglik()
        log(f"converged: sweep {t - 1}, log joint {out['lls'][t - 1]:.6e}, "
            f"{(time.perf_counter() - w0) / (t - 11) * 1e3:.1f} ms per replayed sweep")
    out["replayed_ms_per_sweep"] = (time.perf_counter() - w0) / (901 - 11) * 1e3
    log("converged: sweeps 901-1000")
    out["converged"] = window(901, 100)
    out["lls"][1000] = plan.loglik()
    log(f"converged: last window {out['converged']}")
    plan.set_graph(False)
    plan.phi_step(1001)
    if not args.no_foldin:
        out["foldin"] = foldin_bench(args, torch, pulda, synth, model=plan,
                                     phi_source="Phi-step of sweep 1001 of a 1000-sweep run on the large corpus "
                                                "(seed %d)" % args.seed)
    return out


def alg1_bench(plan, t, N, sweeps):
    """Algorithm 1 (Phi-step phi_k ~ Dir(n_k + beta) by Gamma draws) on the
    state the timed sweeps left, with the same z-step schedule: per-phase
    times from hipEvents, beside the Polya-urn figures of the main run."""
    plan.set_graph(False)
    plan.set_timing(True)
    plan.set_phi_method("dirichlet")
    plan.stats()
    plan.sweep(t, sweeps, want_ll=False)
    st = plan.stats()
    plan.set_phi_method("polya_urn")
    z_ms = st["ms_z"] / st["n_z"]
    return dict(sweeps=sweeps, phi_ms=st["ms_phi"] / st["n_phi"], z_ms=z_ms, z_tokens_per_s=N / (z_ms * 1e-3),
                mean_J=st["sum_J"] / st["z_steps"] / N, a_fraction=st["sum_A"] / st["z_steps"] / N,
                nnz_phi=st["nnz_phi"], fp64_fallbacks_per_token=st["fallback_draws"] / st["z_steps"] / N)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="large", choices=["tiny", "small", "medium", "large"])
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--side-ratio", type=int, default=1, help="side ratio with --force-group")
    ap.add_argument("--separate-loglik", action="store_true",
                    help="recount document terms of the log joint in their own pass")
    ap.add_argument("--schedule", default=None,
                    help="explicit schedule as JSON [min_len, group, docs_per_item, side_ratio] (no autotuning)")
    ap.add_argument("--force-group", type=int, default=0,
                    help="one schedule bucket with this group size (1, 8, 16, 32, 64) instead of autotuning")
    ap.add_argument("--graph", action="store_true", help="replay a captured sweep (no per-phase events)")
    ap.add_argument("--graph-steps", type=int, default=10,
                    help="after the timed sweeps, this many sweeps replayed from a captured graph (0: none)")
    ap.add_argument("--cpu-docs", type=int, default=200000,
                    help="documents of the oracle's z-step baseline (about 10 s of one core at the large config)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-foldin", action="store_true")
    ap.add_argument("--heldout-docs", type=int, default=2000,
                    help="new documents for the held-out log-likelihood (0: none)")
    ap.add_argument("--heldout-max-len", type=int, default=500)
    ap.add_argument("--particles", type=int, default=10)
    ap.add_argument("--heldout-oracle-docs", type=int, default=6)
    ap.add_argument("--scaling", action="store_true",
                    help="run only the scaling study of both Phi-steps on restrictions of the large corpus "
                         "(read from --corpus-cache when present)")
    ap.add_argument("--ksweep", action="store_true",
                    help="run only the K = 10, 100, 1000 comparison of both Phi-steps with log-joint traces")
    ap.add_argument("--trace-sweeps", type=int, default=200, help="sweeps of each log-joint trace in --ksweep")
    ap.add_argument("--ks", type=int, nargs="*", default=[10, 100, 1000], help="topic counts of --ksweep")
    ap.add_argument("--converged", action="store_true",
                    help="run only the 1000-sweep large run (sweeps 1-10 and 901-1000 timed) and fold-in serving "
                         "on its Phi")
    ap.add_argument("--alg1-sweeps", type=int, default=3,
                    help="sweeps with Algorithm 1's Dirichlet Phi-step after the timed region (0: none)")
    ap.add_argument("--foldin-requests", type=int, default=450000,
                    help="requests drawn for the fold-in traces (open-loop traces use what trace_s needs)")
    ap.add_argument("--closed-requests", type=int, default=12000, help="requests of the closed-loop run")
    ap.add_argument("--trace-s", type=float, default=10.0, help="seconds of Poisson arrivals per rate point")
    ap.add_argument("--plain-requests", type=int, default=60)
    ap.add_argument("--foldin-cpu-requests", type=int, default=200,
                    help="requests of the oracle's fold-in baseline (0: none)")
    ap.add_argument("--slots", type=int, default=4096)
    ap.add_argument("--draws", type=int, default=2048, help="fold-in token draws per request per step")
    ap.add_argument("--foldin-group", type=int, default=64, choices=[16, 32, 64], help="lanes per fold-in request")
    ap.add_argument("--rates", type=float, nargs="*", default=[0.5, 0.8, 0.95])
    ap.add_argument("--corpus-cache", default=None,
                    help=".npz file: load the corpus from it if present, else generate and save it there")
    ap.add_argument("--generate-only", action="store_true", help="generate (and cache) the corpus, then exit")
    ap.add_argument("--calibrate", action="store_true",
                    help="first copy 1 GiB device-to-device 3 times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    from paper_1704_03581_amd import synth
    if args.ksweep:
        import torch
        from paper_1704_03581_amd import pulda
        print(json.dumps(dict(metric="K sweep: Phi-step and z-step ms per sweep, Polya urn vs Dirichlet, and "
                                     "log-joint traces", **ksweep_study(args, torch, pulda, synth))), flush=True)
        return
    if args.converged:
        import torch
        from paper_1704_03581_amd import pulda
        print(json.dumps(dict(metric="converged z-step throughput (sweeps 901-1000) and fold-in serving on the "
                                     "converged Phi", **converged_study(args, torch, pulda, synth))), flush=True)
        return
    if args.scaling:
        import torch
        from paper_1704_03581_amd import pulda
        print(json.dumps(dict(metric="scaling study: Phi-step and z-step ms per sweep, Polya urn vs Dirichlet",
                              **scaling_study(args, torch, pulda, synth))), flush=True)
        return
    t0 = time.perf_counter()
    if args.corpus_cache and os.path.exists(args.corpus_cache):
        log(f"loading the {args.config} corpus from {args.corpus_cache}")
        corpus = synth.load(args.corpus_cache)
        assert corpus.name == args.config, (corpus.name, args.config)
    else:
        log(f"generating the {args.config} corpus")
        corpus = synth.generate(args.config, keep_true_z=False)
        if args.corpus_cache:
            synth.save(corpus, args.corpus_cache)
    if args.generate_only:
        return
    log(f"corpus: D={corpus.D} V={corpus.V} K={corpus.K} N={corpus.N} ({time.perf_counter() - t0:.1f}s)")

    import torch
    from paper_1704_03581_amd import pulda
    dev = torch.device("cuda:0")
    if args.calibrate:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("calibration copies: 3 x 1 GiB device-to-device")
    plan = pulda.Plan(corpus.K, corpus.V, corpus.D, corpus.N, alpha=corpus.alpha, beta=corpus.beta,
                      seed=args.seed, device=dev)
    plan.upload(corpus.doc_off, corpus.words)
    plan.init()
    plan.set_fused_loglik(not args.separate_loglik)
    t = 1
    log(f"warmup {args.warmup} sweeps")
    if args.warmup:
        plan.sweep(t, args.warmup, want_ll=False)
        t += args.warmup
    torch.cuda.synchronize()
    # the schedule is tuned on the state the timed sweeps start from
    if args.schedule:
        plan.set_schedule(*json.loads(args.schedule))
        log(f"schedule: {plan.get_schedule()}")
    elif args.force_group:
        plan.set_schedule([0], [args.force_group], [64 // args.force_group * 16], [args.side_ratio])
        log(f"schedule: one bucket, group {args.force_group}, side ratio {args.side_ratio}")
    elif not args.no_autotune:
        plan.phi_step(t)
        sched = plan.autotune(t, reps=1)
        log(f"autotuned schedule: {sched}")
    plan.set_graph(args.graph)
    plan.set_timing(not args.graph)
    torch.cuda.synchronize()
    plan.stats()  # restart counters and event totals
    log(f"timing {args.steps} sweeps")
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    plan.sweep(t, args.steps, want_ll=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    st = plan.stats()
    ll = plan.loglik()
    N = corpus.N
    ms_step = wall * 1e3 / args.steps
    tokens_per_s = N * args.steps / wall
    res = dict(metric="z-step tokens/sec at K=1000 (% HBM roofline); fold-in docs/sec + p50/p99 latency",
               value=tokens_per_s, unit="tokens/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=ms_step, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32+f64",
               data="synthetic",
               config=dict(workload=f"{args.config}: synthetic LDA corpus D={corpus.D} V={corpus.V} K={corpus.K} "
                                    f"N={N}, alpha={corpus.alpha}, beta={corpus.beta}; one sweep = Phi-step + "
                                    f"z-step + count rebuild + log joint",
                           global_batch=N, parallelism="single GPU", schedule=plan.get_schedule()))
    if not args.graph and st["n_z"]:
        z_ms = st["ms_z"] / st["n_z"]
        bytes_launch = algorithmic_bytes(N, st["sum_J"] / st["z_steps"], st["sum_A"] / st["z_steps"])
        # the same with the b-terms of the tokens whose b-part was computed
        # (a token whose a-part is certain at staging reads none of its J)
        bytes_b = algorithmic_bytes(N, st["sum_J_b"] / st["z_steps"], st["sum_A"] / st["z_steps"])
        achieved = bytes_launch / (z_ms * 1e-3) / 1e9
        res["zstep"] = dict(tokens_per_s=N / (z_ms * 1e-3), kernel_ms=z_ms, phi_ms=st["ms_phi"] / st["n_phi"],
                            loglik_ms=st["ms_ll"] / st["n_ll"],
                            mean_J=st["sum_J"] / st["z_steps"] / N, a_fraction=st["sum_A"] / st["z_steps"] / N,
                            degenerate_per_sweep=st["degenerate_tokens"] / st["z_steps"],
                            nnz_phi=st["nnz_phi"], loglik=ll)
        traffic, tsrc = recorded_traffic(args.config)
        res["roofline"] = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                               frac=achieved / HBM_PEAK_GBS, traffic=traffic,
                               kernel="z_step_kernel", algorithmic_bytes_per_launch=bytes_launch,
                               frac_b_terms_read=bytes_b / (z_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                               algorithmic_bytes_b_terms_read=bytes_b,
                               frac_rocprof=(traffic / (z_ms * 1e-3) / 1e9 / HBM_PEAK_GBS) if traffic else None,
                               target_frac=0.40, target_met=achieved / HBM_PEAK_GBS >= 0.40,
                               traffic_unit="bytes per launch (FETCH_SIZE x2.0 + WRITE_SIZE x1.0, calibrated)",
                               traffic_source=os.path.relpath(tsrc, ROOT) if tsrc else None)
        res["zstep"]["mean_J_b_terms_read"] = st["sum_J_b"] / st["z_steps"] / N
        # draws whose fp32 b-part was too close to a boundary to decide
        res["zstep"]["fp64_fallbacks_per_token"] = st["fallback_draws"] / st["z_steps"] / N
    log(f"sweep {ms_step:.2f} ms, {tokens_per_s / 1e9:.3f} G tokens/s; {res.get('zstep')}")
    t = t + args.steps
    if not args.graph and args.graph_steps > 0:
        # the same sweeps replayed from a captured hipGraph (no per-phase
        # events), timed by the host clock
        plan.set_timing(False)
        plan.set_graph(True)
        plan.sweep(t, 1, want_ll=False)      # capture
        t += 1
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        plan.sweep(t, args.graph_steps, want_ll=False)
        torch.cuda.synchronize()
        gwall = time.perf_counter() - g0
        t += args.graph_steps
        plan.set_graph(False)
        res["graph"] = dict(steps=args.graph_steps, ms_per_step=gwall * 1e3 / args.graph_steps,
                            tokens_per_s=N * args.graph_steps / gwall)
        log(f"graph replay: {res['graph']}")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_baseline(corpus, args.seed, args.cpu_docs)
    ho_docs = None
    if args.heldout_docs > 0:
        log(f"held-out log-likelihood of {args.heldout_docs} new documents (urn Phi)")
        ho_docs = synth.foldin_requests(args.heldout_docs, seed=170403581 + 6, base=args.config,
                                        max_len=args.heldout_max_len)
        plan.heldout_loglik(ho_docs[:2], particles=2, seed=args.seed)   # load the kernels
        res["heldout"] = dict(
            workload=f"{args.heldout_docs} new documents of the fold-in length law up to {args.heldout_max_len} "
                     f"tokens, words from the generating Phi; left-to-right estimate, {args.particles} particles",
            polya_urn=heldout_bench(plan, ho_docs, args.particles, args.seed, torch,
                                    oracle_docs=0 if args.no_cpu_baseline else args.heldout_oracle_docs,
                                    K=corpus.K, V=corpus.V, alpha=corpus.alpha))
        log(f"heldout {res['heldout']['polya_urn']}")
    if args.alg1_sweeps > 0:
        log(f"Algorithm 1 (Dirichlet Phi-step): {args.alg1_sweeps} sweeps")
        res["alg1"] = alg1_bench(plan, t, N, args.alg1_sweeps)
        if "zstep" in res:
            res["alg1"]["phi_speedup_polya_urn"] = res["alg1"]["phi_ms"] / res["zstep"]["phi_ms"]
            res["alg1"]["z_speedup_polya_urn"] = res["alg1"]["z_ms"] / res["zstep"]["kernel_ms"]
        log(f"alg1 {res['alg1']}")
        if ho_docs is not None:
            res["heldout"]["dirichlet"] = heldout_bench(plan, ho_docs, args.particles, args.seed, torch)
            log(f"heldout (Dirichlet Phi) {res['heldout']['dirichlet']}")
    del plan
    torch.cuda.empty_cache()
    if not args.no_foldin:
        res["foldin"] = foldin_bench(args, torch, pulda, synth)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
