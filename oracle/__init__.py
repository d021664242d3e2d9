"""CPU oracle for the Polya-urn LDA sampler -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The sampler itself never calls it.

A thin ctypes/numpy wrapper over ``pulda_oracle.c`` (plain single-threaded C,
fp64, ``-ffp-contract=off``).  Every function names the part of the paper it
follows in the C source.  Arrays follow the paper's K x V orientation
(``n[k, v]``, ``phi[k, v]``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pulda_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

TAG_INIT, TAG_PHI_CELL, TAG_PHI_PRIOR, TAG_Z, TAG_FOLDIN_INIT, TAG_FOLDIN_Z, TAG_PHI_GAMMA, TAG_LTR = range(8)


def build() -> str:
    """Compile the oracle (always; cheap)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


P = C.POINTER
u8p, u16p, u32p, i32p, i64p, f32p, f64p = (P(C.c_uint8), P(C.c_uint16), P(C.c_uint32), P(C.c_int32),
                                          P(C.c_int64), P(C.c_float), P(C.c_double))


def _declare(L):
    L.or_philox.argtypes = [u32p, u32p, u32p]
    L.or_vose.argtypes = [f64p, C.c_int32, u32p, i32p]
    L.or_pois_support.argtypes = [C.c_double, C.c_int32]
    L.or_pois_support.restype = C.c_int32
    L.or_pois_table.argtypes = [C.c_double, C.c_int32, u32p, i32p]
    L.or_ztp_thresholds.argtypes = [C.c_double, u32p, C.c_int32]
    L.or_ztp_thresholds.restype = C.c_int32
    L.or_init_z.argtypes = [C.c_int64, C.c_int32, C.c_uint64, u16p]
    L.or_counts.argtypes = [C.c_int64, C.c_int32, C.c_int32, i64p, i32p, u16p, i32p, i64p, i32p]
    L.or_phi_counts.argtypes = [C.c_int32, C.c_int32, C.c_double, f64p, C.c_int32, C.c_uint64, C.c_uint32, i32p,
                                i32p]
    L.or_phi_normalise.argtypes = [C.c_int32, C.c_int32, i32p, i64p, f32p]
    L.or_phi_normalise.restype = C.c_int32
    L.or_gamma_draw.argtypes = [C.c_double, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32]
    L.or_gamma_draw.restype = C.c_double
    L.or_phi_dirichlet.argtypes = [C.c_int32, C.c_int32, C.c_double, f64p, C.c_uint64, C.c_uint32, i32p, f64p, f64p,
                                   f32p]
    L.or_phi_dirichlet.restype = C.c_int32
    L.or_word_tables.argtypes = [C.c_int32, C.c_int32, f64p, f32p, i64p, u16p, f32p, u32p, u16p, f64p]
    L.or_word_tables.restype = C.c_int64
    L.or_z_step.argtypes = [C.c_int64, C.c_int32, C.c_int32, i64p, i32p, u16p, C.c_uint64, C.c_uint32, f32p,
                            i64p, u16p, u32p, u16p, f64p, i64p]
    L.or_z_step.restype = C.c_int64
    L.or_z_step_sparse.argtypes = L.or_z_step.argtypes
    L.or_z_step_sparse.restype = C.c_int64
    L.or_replay.argtypes = [C.c_int64, C.c_int32, C.c_int32, i64p, i32p, u16p, u16p, C.c_uint64, C.c_uint32,
                            f32p, i64p, u16p, u32p, u16p, f64p, C.c_double, i64p, f64p, i64p, i64p, C.c_int64]
    L.or_loglik.argtypes = [C.c_int64, C.c_int32, C.c_int32, i64p, i32p, u16p, f64p, C.c_double, f64p]
    L.or_loglik.restype = C.c_double
    L.or_foldin.argtypes = [C.c_int32, C.c_int32, f32p, i64p, u16p, u32p, u16p, f64p, f64p, C.c_uint64,
                            C.c_uint32, i32p, C.c_int32, C.c_int32, C.c_int32, f32p, f64p, i32p, u16p]
    L.or_foldin.restype = C.c_int32
    L.or_heldout_ltr.argtypes = [C.c_int32, C.c_int32, f32p, i64p, u16p, u32p, u16p, f64p, f64p, C.c_uint64,
                                 C.c_uint32, i32p, C.c_int32, C.c_int32, f64p, i32p]
    L.or_heldout_ltr.restype = C.c_double
    L.or_token_pmf.argtypes = [C.c_int32, C.c_int32, f32p, i64p, u16p, u32p, u16p, f64p, C.c_int32, i32p,
                               f64p, f64p]


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def philox(ctr, key):
    ctr = _c(ctr, np.uint32)
    key = _c(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox(_p(ctr, C.c_uint32), _p(key, C.c_uint32), _p(out, C.c_uint32))
    return out


def vose(w):
    w = _c(w, np.float64)
    n = len(w)
    thr = np.zeros(n, np.uint32)
    alias = np.zeros(n, np.int32)
    lib().or_vose(_p(w, C.c_double), n, _p(thr, C.c_uint32), _p(alias, C.c_int32))
    return thr, alias


def pois_table(beta, l):
    n = lib().or_pois_support(beta, l)
    thr = np.zeros(n, np.uint32)
    alias = np.zeros(n, np.int32)
    lib().or_pois_table(beta, l, _p(thr, C.c_uint32), _p(alias, C.c_int32))
    return thr, alias


def ztp_thresholds(beta, cap=64):
    """Zero-truncated Pois(beta) thresholds floor(2^32 P(X <= x | X >= 1)),
    x = 1.., at least 5, up to the first that saturates."""
    T = np.zeros(cap, np.uint32)
    n = lib().or_ztp_thresholds(beta, _p(T, C.c_uint32), cap)
    return T[:n].copy()


def _beta_arg(beta_v, V):
    if beta_v is None:
        return None, None
    b = _c(np.broadcast_to(beta_v, (V,)), np.float64)
    return b, _p(b, C.c_double)


def init_z(N, K, seed):
    z = np.zeros(N, np.uint16)
    lib().or_init_z(N, K, seed, _p(z, C.c_uint16))
    return z


def counts(doc_off, words, z, K, V, with_m=True):
    doc_off = _c(doc_off, np.int64)
    words = _c(words, np.int32)
    z = _c(z, np.uint16)
    D = len(doc_off) - 1
    n = np.zeros((K, V), np.int32)
    nk = np.zeros(K, np.int64)
    m = np.zeros((D, K), np.int32) if with_m else None
    lib().or_counts(D, K, V, _p(doc_off, C.c_int64), _p(words, C.c_int32), _p(z, C.c_uint16),
                    _p(n, C.c_int32), _p(nk, C.c_int64), _p(m, C.c_int32) if with_m else None)
    return n, nk, m


def phi_counts(n, beta, L, seed, t, beta_v=None):
    """Poisson draws of the Polya-urn Phi-step; beta_v: V priors (or None:
    the symmetric beta)."""
    n = _c(n, np.int32)
    K, V = n.shape
    gam = np.zeros((K, V), np.int32)
    keep, bp = _beta_arg(beta_v, V)
    lib().or_phi_counts(K, V, beta, bp, L, seed, t, _p(n, C.c_int32), _p(gam, C.c_int32))
    return gam


def phi_normalise(gam):
    gam = _c(gam, np.int32)
    K, V = gam.shape
    S = np.zeros(K, np.int64)
    phi = np.zeros((K, V), np.float32)
    empty = lib().or_phi_normalise(K, V, _p(gam, C.c_int32), _p(S, C.c_int64), _p(phi, C.c_float))
    return S, phi, empty


def gamma_draw(a, seed, c0, c1, c2):
    """One G(a, 1) draw of Algorithm 1's Phi-step (Marsaglia-Tsang) at
    Philox counter (c0, c1, c2, PHI_GAMMA + 256 j)."""
    return lib().or_gamma_draw(float(a), seed, c0, c1, c2)


def phi_dirichlet(n, beta, seed, t, beta_v=None):
    """Algorithm 1's Phi-step: phi_k ~ Dir(n_k + beta) via Gamma draws.
    Returns (gamma fp64 K x V, S fp64 K, phi fp32 K x V, empty rows)."""
    n = _c(n, np.int32)
    K, V = n.shape
    keep, bp = _beta_arg(beta_v, V)
    gam = np.zeros((K, V), np.float64)
    S = np.zeros(K, np.float64)
    phi = np.zeros((K, V), np.float32)
    empty = lib().or_phi_dirichlet(K, V, beta, bp, seed, t, _p(n, C.c_int32), _p(gam, C.c_double),
                                   _p(S, C.c_double), _p(phi, C.c_float))
    return gam, S, phi, empty


@dataclass
class WordTables:
    colptr: np.ndarray       # int64[V+1]
    topic: np.ndarray        # uint16[nnz]
    phi: np.ndarray          # float32[nnz]
    thr: np.ndarray          # uint32[nnz]
    alias_topic: np.ndarray  # uint16[nnz]
    sigma_a: np.ndarray      # float64[V]


def word_tables(alpha, phi):
    phi = _c(phi, np.float32)
    K, V = phi.shape
    alpha = _c(np.broadcast_to(alpha, (K,)), np.float64)
    nnz = lib().or_word_tables(K, V, _p(alpha, C.c_double), _p(phi, C.c_float), None, None, None, None, None, None)
    colptr = np.zeros(V + 1, np.int64)
    topic = np.zeros(nnz, np.uint16)
    ph = np.zeros(nnz, np.float32)
    thr = np.zeros(nnz, np.uint32)
    at = np.zeros(nnz, np.uint16)
    sa = np.zeros(V, np.float64)
    lib().or_word_tables(K, V, _p(alpha, C.c_double), _p(phi, C.c_float), _p(colptr, C.c_int64),
                         _p(topic, C.c_uint16), _p(ph, C.c_float), _p(thr, C.c_uint32), _p(at, C.c_uint16),
                         _p(sa, C.c_double))
    return WordTables(colptr, topic, ph, thr, at, sa)


def _model_args(phi, wt):
    return (_p(phi, C.c_float), _p(wt.colptr, C.c_int64), _p(wt.topic, C.c_uint16), _p(wt.thr, C.c_uint32),
            _p(wt.alias_topic, C.c_uint16), _p(wt.sigma_a, C.c_double))


def z_step(doc_off, words, z, seed, t, phi, wt, K, V, sparse=False):
    """One z-step.  Returns (new z, degenerate count, sum_J, sum_A).

    sparse=False walks every topic per token (the plain definition);
    sparse=True iterates the smaller of the document's topics and the word's
    Phi column, with the same results bit for bit (the timed CPU mode)."""
    doc_off = _c(doc_off, np.int64)
    words = _c(words, np.int32)
    z = np.array(z, dtype=np.uint16, copy=True)
    phi = _c(phi, np.float32)
    stats = np.zeros(2, np.int64)
    fn = lib().or_z_step_sparse if sparse else lib().or_z_step
    deg = fn(len(doc_off) - 1, K, V, _p(doc_off, C.c_int64), _p(words, C.c_int32),
             _p(z, C.c_uint16), seed, t, *_model_args(phi, wt), _p(stats, C.c_int64))
    return z, int(deg), int(stats[0]), int(stats[1])


def replay(doc_off, words, z_before, z_after, seed, t, phi, wt, K, V, tol=1e-6, docs=None):
    """Teacher-forced check of another implementation's z-step.

    Returns dict(agree, ties, bad, degenerate, worst_rel, first_bad).  With
    ``docs`` only those documents are checked."""
    doc_off = _c(doc_off, np.int64)
    words = _c(words, np.int32)
    zb = _c(z_before, np.uint16)
    za = _c(z_after, np.uint16)
    phi = _c(phi, np.float32)
    out = np.zeros(4, np.int64)
    worst = np.zeros(1, np.float64)
    first = np.zeros(1, np.int64)
    dl = None if docs is None else _c(docs, np.int64)
    lib().or_replay(len(doc_off) - 1, K, V, _p(doc_off, C.c_int64), _p(words, C.c_int32), _p(zb, C.c_uint16),
                    _p(za, C.c_uint16), seed, t, *_model_args(phi, wt), tol, _p(out, C.c_int64),
                    _p(worst, C.c_double), _p(first, C.c_int64),
                    _p(dl, C.c_int64) if dl is not None else None, 0 if dl is None else len(dl))
    return dict(agree=int(out[0]), ties=int(out[1]), bad=int(out[2]), degenerate=int(out[3]),
                worst_rel=float(worst[0]), first_bad=int(first[0]))


def loglik(doc_off, words, z, alpha, beta, K, V, beta_v=None):
    doc_off = _c(doc_off, np.int64)
    words = _c(words, np.int32)
    z = _c(z, np.uint16)
    alpha = _c(np.broadcast_to(alpha, (K,)), np.float64)
    keep, bp = _beta_arg(beta_v, V)
    return float(lib().or_loglik(len(doc_off) - 1, K, V, _p(doc_off, C.c_int64), _p(words, C.c_int32),
                                 _p(z, C.c_uint16), _p(alpha, C.c_double), beta, bp))


def foldin(phi, wt, alpha, seed, req, words, S=50, burn_in=25):
    """Fold-in of one request; returns (theta fp32[K], loglik, kept, dropped, z_final)."""
    phi = _c(phi, np.float32)
    K, V = phi.shape
    alpha = _c(np.broadcast_to(alpha, (K,)), np.float64)
    words = _c(words, np.int32)
    theta = np.zeros(K, np.float32)
    ll = np.zeros(1, np.float64)
    dropped = np.zeros(1, np.int32)
    zf = np.zeros(max(len(words), 1), np.uint16)
    if S <= burn_in:
        raise ValueError("S must exceed burn_in")
    kept = lib().or_foldin(K, V, *_model_args(phi, wt), _p(alpha, C.c_double), seed, req, _p(words, C.c_int32),
                           len(words), S, burn_in, _p(theta, C.c_float), _p(ll, C.c_double),
                           _p(dropped, C.c_int32), _p(zf, C.c_uint16))
    return theta, float(ll[0]), int(kept), int(dropped[0]), zf[:len(words)]


def token_pmf(phi, wt, v, m):
    """Exhaustive enumeration of one token draw over all 2^24 values of u.

    Returns (mass_b[K], mass_a): the b-part law and the a-part's total mass."""
    phi = _c(phi, np.float32)
    K, V = phi.shape
    m = _c(m, np.int32)
    mb = np.zeros(K, np.float64)
    ma = np.zeros(1, np.float64)
    lib().or_token_pmf(K, V, *_model_args(phi, wt), v, _p(m, C.c_int32), _p(mb, C.c_double), _p(ma, C.c_double))
    return mb, float(ma[0])


class Sampler:
    """Algorithm 2 end to end on the CPU: Phi-step then z-step per sweep."""

    def __init__(self, doc_off, words, K, V, alpha=0.1, beta=0.01, L=100, seed=1, z0=None, sparse=False):
        self.doc_off = _c(doc_off, np.int64)
        self.words = _c(words, np.int32)
        self.K, self.V = K, V
        self.alpha = _c(np.broadcast_to(alpha, (K,)), np.float64)
        self.beta, self.L, self.seed, self.sparse = beta, L, seed, sparse
        N = int(self.doc_off[-1])
        self.z = init_z(N, K, seed) if z0 is None else np.array(z0, dtype=np.uint16, copy=True)
        self.n, self.nk, _ = counts(self.doc_off, self.words, self.z, K, V, with_m=False)

    def phi_step(self, t):
        self.gam = phi_counts(self.n, self.beta, self.L, self.seed, t)
        self.S, self.phi, self.empty_rows = phi_normalise(self.gam)
        self.wt = word_tables(self.alpha, self.phi)

    def z_step(self, t):
        self.z_prev = self.z
        self.z, self.degenerate, self.sum_J, self.sum_A = z_step(
            self.doc_off, self.words, self.z, self.seed, t, self.phi, self.wt, self.K, self.V, sparse=self.sparse)
        self.n, self.nk, _ = counts(self.doc_off, self.words, self.z, self.K, self.V, with_m=False)

    def loglik(self):
        return loglik(self.doc_off, self.words, self.z, self.alpha, self.beta, self.K, self.V)

    def sweep(self, t):
        self.phi_step(t)
        self.z_step(t)
        return self.loglik()


def heldout_ltr(phi, wt, alpha, seed, req, words, R, want_Z=False):
    """Left-to-right held-out estimate of log p(words | Phi, alpha) with R
    particles.  Returns (estimate, kept tokens[, Z (R x kept)])."""
    phi = _c(phi, np.float32)
    K, V = phi.shape
    alpha = _c(np.broadcast_to(alpha, (K,)), np.float64)
    words = _c(words, np.int32)
    kept = C.c_int32()
    # R x kept values, row stride = kept (at most R x len)
    Zs = np.zeros(R * max(len(words), 1), np.float64) if want_Z else None
    ll = lib().or_heldout_ltr(K, V, *_model_args(phi, wt), _p(alpha, C.c_double), seed, req, _p(words, C.c_int32),
                              len(words), R, _p(Zs, C.c_double) if want_Z else None, C.byref(kept))
    if want_Z:
        return ll, kept.value, Zs[:R * kept.value].reshape(R, kept.value).copy()
    return ll, kept.value
