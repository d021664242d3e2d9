"""Pins of the oracle's teacher-forced replay and of its sparse z-step mode
(CPU only).

The replay decides every z-step parity test: it redraws each token from the
other side's preceding draws and sorts a disagreement into a tie (x within
tol * Z of the x-values that give the other side's topic) or a failure.  The
tests below feed it states whose classification is known from outside the
oracle: the oracle's own draws (all agree), a topic whose b-term is zero and
which the alias slot cannot give (a failure at any tolerance), values that
are not topics, and constructed ties, where a Phi value is solved for so that
a boundary of the token's conditional (Section 3.5: sigma_a between the a-
and b-parts, a running b-sum between two topics) lies a known tiny distance
from x.  The boundary and x are recomputed here in fp64 with the definition's
order of sums, independently of the oracle's code.

The sparse mode iterates the smaller of the document's topics and the word's
Phi column (Section 3.5; cost in Section 3.6); it must reproduce the dense
plain definition bit for bit.
"""
import numpy as np
import pytest

import oracle

K4 = 4
ALPHA = 0.1


def _u24(r0):
    return float(int(r0) >> 8) * (1.0 / 16777216.0)


def _token_r(seed, i, t):
    return oracle.philox(np.array([i & 0xFFFFFFFF, i >> 32, t, oracle.TAG_Z], np.uint32),
                         np.array([seed & 0xFFFFFFFF, seed >> 32], np.uint32))


def _tables(p):
    """One word (V = 1), K = 4 topics with column values p (fp32)."""
    phi = np.asarray(p, np.float32).reshape(K4, 1)
    wt = oracle.word_tables(np.full(K4, ALPHA), phi)
    return phi, wt


def _boundaries(phi, wt, m):
    """x-value boundaries of the token conditional with counts m: sigma_a,
    then the running sums sigma_a + b_1 + ... over topics with b_k > 0 in
    ascending order (fp64, the definition's order).  Returns (sa, Z, list of
    (topic, lo, hi))."""
    sa = float(wt.sigma_a[0])
    sb = 0.0
    for k in range(K4):
        sb += float(phi[k, 0]) * float(m[k])
    Z = sa + sb
    iv = []
    c = sa
    for k in range(K4):
        b = float(phi[k, 0]) * float(m[k])
        if b > 0.0:
            iv.append((k, c, c + b))
            c = c + b
    return sa, Z, iv


def _alias_draw(wt, r):
    n = int(wt.colptr[1] - wt.colptr[0])
    j = (int(r[1]) * n) >> 32
    return int(wt.topic[j]) if int(r[2]) < int(wt.thr[j]) else int(wt.alias_topic[j])


def _draw_py(seed, i, m, phi, wt):
    """Token i's draw with counts m, from the definition (Section 3.5)."""
    r = _token_r(seed, i, T)
    sa, Z, iv = _boundaries(phi, wt, m)
    x = _u24(r[0]) * Z
    if x < sa:
        return _alias_draw(wt, r)
    for k, lo, hi in iv:
        if x < hi:
            return k
    return iv[-1][0]


def _teacher_forced(seed, first, phi, wt):
    """The document's draws when token 0 is `first`: each later token drawn
    from the counts of the earlier draws and the later tokens' old topics."""
    z = [first]
    for i in range(1, 3):
        m = np.bincount(np.array(z + list(Z_BEFORE[i + 1:]), np.int64), minlength=K4)
        z.append(_draw_py(seed, i, m, phi, wt))
    return np.array(z, np.uint16)


# one document of three tokens of word 0 with topics 0, 1, 2: token 0 is
# drawn with m^{-0} = {1: 1, 2: 1}
DOC_OFF = np.array([0, 3], np.int64)
WORDS = np.zeros(3, np.int32)
Z_BEFORE = np.array([0, 1, 2], np.uint16)
M_TOKEN0 = np.array([0, 1, 1, 0])
T = 7


def _oracle_after(seed, phi, wt):
    z, _, _, _ = oracle.z_step(DOC_OFF, WORDS, Z_BEFORE, seed, T, phi, wt, K4, 1)
    return z


def test_replay_own_draws_agree():
    rng = np.random.default_rng(3)
    for seed in range(1, 6):
        phi, wt = _tables(rng.uniform(0.05, 1.0, K4))
        za = _oracle_after(seed, phi, wt)
        r = oracle.replay(DOC_OFF, WORDS, Z_BEFORE, za, seed, T, phi, wt, K4, 1)
        assert r == dict(agree=3, ties=0, bad=0, degenerate=0, worst_rel=0.0, first_bad=-1), r


def test_replay_wrong_topic_is_bad():
    # topic 3 has a zero b-term for token 0 (m_3 = 0); with phi_3 = 0 the
    # alias table cannot give it either, so no x yields it
    phi, wt = _tables([0.3, 0.4, 0.5, 0.0])
    for seed in range(1, 6):
        za = _oracle_after(seed, phi, wt)
        bad = za.copy()
        bad[0] = 3
        r = oracle.replay(DOC_OFF, WORDS, Z_BEFORE, bad, seed, T, phi, wt, K4, 1, tol=1e-3)
        assert r["bad"] >= 1 and r["first_bad"] == 0, r
        assert r["worst_rel"] == np.inf


def test_replay_wrong_neighbour_far_from_boundary_is_bad():
    # the last token of the document: no later token depends on it.  The
    # other side claims a b-topic whose interval is far from x: bad, and the
    # reported distance is that to the claimed interval
    phi, wt = _tables([0.3, 0.4, 0.5, 0.2])
    checked = 0
    for seed in range(1, 200):
        za = _oracle_after(seed, phi, wt)
        i = 2
        m = np.bincount(za[:i].astype(np.int64), minlength=K4) + np.bincount(Z_BEFORE[i + 1:].astype(np.int64),
                                                                            minlength=K4)
        sa, Z, iv = _boundaries(phi, wt, m)
        r = _token_r(seed, i, T)
        x = _u24(r[0]) * Z
        if x < sa:
            continue
        mine = [k for k, lo, hi in iv if lo <= x < hi]
        others = [(k, lo, hi) for k, lo, hi in iv if k not in mine and k != _alias_draw(wt, r)]
        if not mine or not others:
            continue
        k, lo, hi = others[0]
        want = (lo - x if x < lo else x - hi) / Z
        if want < 1e-3:
            continue
        z2 = za.copy()
        z2[i] = k
        out = oracle.replay(DOC_OFF, WORDS, Z_BEFORE, z2, seed, T, phi, wt, K4, 1)
        assert out["bad"] == 1 and out["agree"] == 2 and out["first_bad"] == i, out
        assert abs(out["worst_rel"] - want) <= 1e-12, (out, want)
        checked += 1
        if checked >= 5:
            break
    assert checked >= 5


def test_replay_values_that_are_not_topics():
    phi, wt = _tables([0.3, 0.4, 0.5, 0.2])
    za = _oracle_after(1, phi, wt)
    z2 = za.copy()
    z2[1] = 0xFFFF   # the padding value of the kernels' topic lists
    r = oracle.replay(DOC_OFF, WORDS, Z_BEFORE, z2, 1, T, phi, wt, K4, 1)
    assert r["bad"] >= 1 and r["first_bad"] == 1 and r["worst_rel"] == np.inf, r
    z2[1] = K4       # the first value past the topics
    r = oracle.replay(DOC_OFF, WORDS, Z_BEFORE, z2, 1, T, phi, wt, K4, 1)
    assert r["bad"] >= 1 and r["first_bad"] == 1, r
    zb = Z_BEFORE.copy()
    zb[2] = 0xFFFF
    r = oracle.replay(DOC_OFF, WORDS, zb, za, 1, T, phi, wt, K4, 1)
    assert r["bad"] == 3 and r["agree"] == 0 and r["first_bad"] == 2, r


def _solve_tie(kind, u):
    """Column values (fp32) that put a boundary of token 0's conditional
    near x = u Z, with p_0 = p_1 = p_3 = 0.25 and p_2 free:
      kind 'b': the boundary between topics 1 and 2, sigma_a + p_1 = u Z;
      kind 'a': the boundary sigma_a = u Z.
    sigma_a = 0.1 (p_0 + ... + p_3), Z = sigma_a + p_1 + p_2."""
    if kind == "b":
        p2 = 0.325 * (1.0 - u) / (1.1 * u - 0.1)
    else:
        p2 = (0.075 - 0.325 * u) / (1.1 * u - 0.1)
    return p2


def _find_tie(kind, lo_rel=2e-9, hi_rel=3e-7):
    """Search seeds and fp32 neighbours of the solved p_2 for a case where x
    lies above the boundary by a relative distance in (lo_rel, hi_rel), so
    the oracle takes the upper side.  Returns (seed, phi, wt, rel, x, B)."""
    for seed in range(1, 400):
        r = _token_r(seed, 0, T)
        u = _u24(r[0])
        if kind == "b" and not 0.3 < u < 0.9:
            continue
        if kind == "a" and not 0.12 < u < 0.2:
            continue
        p2 = np.float32(_solve_tie(kind, u))
        for step in range(-300, 301):
            q = p2
            for _ in range(abs(step)):
                q = np.nextafter(q, np.float32(np.inf if step > 0 else 0), dtype=np.float32)
            phi, wt = _tables([0.25, 0.25, float(q), 0.25])
            sa, Z, iv = _boundaries(phi, wt, M_TOKEN0)
            x = u * Z
            B = sa if kind == "a" else iv[0][2]
            rel = (x - B) / Z
            if lo_rel < rel < hi_rel:
                if kind == "a" and _alias_draw(wt, r) == 1:
                    continue   # the a-part would give the same topic: no disagreement to classify
                return seed, phi, wt, rel, x, B
    raise AssertionError("no constructed tie found")


@pytest.mark.parametrize("kind", ["b", "a"])
def test_replay_constructed_tie(kind):
    seed, phi, wt, rel, x, B = _find_tie(kind)
    za = _oracle_after(seed, phi, wt)
    # the oracle takes the side above the boundary: topic 2 (b) or topic 1,
    # the first b-topic (a)
    assert za[0] == (2 if kind == "b" else 1), za
    assert np.array_equal(za, _teacher_forced(seed, int(za[0]), phi, wt))
    r = _token_r(seed, 0, T)
    # the other side of the boundary: topic 1 (b), or the alias draw (a);
    # the later tokens follow from that state
    other = _teacher_forced(seed, 1 if kind == "b" else _alias_draw(wt, r), phi, wt)
    zb2 = Z_BEFORE.copy()
    tie = oracle.replay(DOC_OFF, WORDS, zb2, other, seed, T, phi, wt, K4, 1, tol=1e-6)
    assert tie["ties"] == 1 and tie["bad"] == 0 and tie["agree"] == 2, tie
    # the reported distance is |x - B| / Z, computed here independently
    assert abs(tie["worst_rel"] - rel) <= 1e-9 * rel + 1e-18, (tie["worst_rel"], rel)
    # just below that distance the same disagreement is a failure, just above a tie
    assert oracle.replay(DOC_OFF, WORDS, zb2, other, seed, T, phi, wt, K4, 1, tol=0.9 * rel)["bad"] == 1
    assert oracle.replay(DOC_OFF, WORDS, zb2, other, seed, T, phi, wt, K4, 1, tol=1.1 * rel)["ties"] == 1


# --------------------------------------------------------------------------
# sparse mode == dense plain definition, bit for bit
# --------------------------------------------------------------------------
def _corpus(rng, D, V, K, mean_len):
    lens = rng.poisson(mean_len, D)
    doc_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    words = rng.integers(0, V, int(doc_off[-1])).astype(np.int32)
    return doc_off, words


@pytest.mark.parametrize("K,V,mean_len,density", [(5, 40, 30, 0.9), (50, 200, 60, 0.3), (300, 500, 120, 0.05),
                                                  (300, 500, 400, 0.6)])
def test_sparse_mode_bit_identical(K, V, mean_len, density):
    rng = np.random.default_rng(K + V)
    doc_off, words = _corpus(rng, 80, V, K, mean_len)
    phi = (rng.uniform(0, 1, (K, V)) * (rng.uniform(0, 1, (K, V)) < density)).astype(np.float32)
    phi[:, 3] = 0   # an empty column: degenerate tokens
    alpha = np.full(K, 0.1)
    wt = oracle.word_tables(alpha, phi)
    z = oracle.init_z(len(words), K, 4)
    sides = 0
    for t in range(1, 4):
        zd, dd, jd, ad = oracle.z_step(doc_off, words, z, 4, t, phi, wt, K, V)
        zs, ds, js, as_ = oracle.z_step(doc_off, words, z, 4, t, phi, wt, K, V, sparse=True)
        assert np.array_equal(zd, zs) and (dd, jd, ad) == (ds, js, as_)
        sides += jd
        z = zd
    assert sides > 0


def test_sparse_sampler_matches_dense_sampler():
    rng = np.random.default_rng(8)
    doc_off, words = _corpus(rng, 60, 300, 40, 80)
    a = oracle.Sampler(doc_off, words, 40, 300, seed=3)
    b = oracle.Sampler(doc_off, words, 40, 300, seed=3, sparse=True)
    for t in range(1, 6):
        assert a.sweep(t) == b.sweep(t)
        assert np.array_equal(a.z, b.z)
