"""Shared helpers of the GPU tests (comparison with the oracle)."""
import numpy as np

import oracle


def say(msg: str):
    print(f"[gpu-test] {msg}", flush=True)


def phi_from_gpu(g: dict, K: int, V: int):
    """Dense phi (K x V float32) and oracle.WordTables from a GPU Phi export."""
    phi = np.zeros((K, V), np.float32)
    colptr = g["colptr"].astype(np.int64)
    cols = np.repeat(np.arange(V), np.diff(colptr))
    phi[g["topic"].astype(np.int64), cols] = g["phi"]
    wt = oracle.WordTables(colptr, g["topic"].astype(np.uint16), g["phi"].astype(np.float32),
                           g["alias_thr"].astype(np.uint32), g["alias_topic"].astype(np.uint16),
                           g["sigma_a"].astype(np.float64))
    return phi, wt


def oracle_phi(doc_off, words, z, K, V, alpha, beta, L, seed, t, beta_v=None):
    n, nk, _ = oracle.counts(doc_off, words, z, K, V, with_m=False)
    gam = oracle.phi_counts(n, beta, L, seed, t, beta_v=beta_v)
    S, phi, empty = oracle.phi_normalise(gam)
    wt = oracle.word_tables(alpha, phi)
    return gam, S, phi, wt


def assert_phi_equal(g: dict, gam, S, phi, wt, K, V):
    assert np.array_equal(g["colptr"], wt.colptr), "column pointers differ"
    assert np.array_equal(g["topic"], wt.topic), "column topics differ"
    cols = np.repeat(np.arange(V), np.diff(wt.colptr))
    assert np.array_equal(g["gamma"], gam[wt.topic.astype(np.int64), cols]), "Poisson draws differ"
    assert np.array_equal(g["S"], S), "row sums differ"
    assert np.array_equal(g["phi"].view(np.uint32), wt.phi.view(np.uint32)), "phi differs"
    assert np.array_equal(g["sigma_a"].view(np.uint64), wt.sigma_a.view(np.uint64)), "sigma_a differs"
    assert np.array_equal(g["alias_thr"], wt.thr), "alias thresholds differ"
    assert np.array_equal(g["alias_topic"], wt.alias_topic), "alias topics differ"
