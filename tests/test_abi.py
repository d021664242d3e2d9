"""The C ABI library loads, exports every declared entry point, and checks
arguments on the host (no GPU needed: nothing here launches a kernel)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pulda.h")
LIB = os.path.join(ROOT, "paper_1704_03581_amd", "libpulda.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pulda_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libpulda.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 30
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_1704_03581_amd import pulda
    assert sorted(pulda.EXPORTED) == declared()


class Desc(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("V", ctypes.c_int32), ("beta", ctypes.c_double), ("alpha", ctypes.c_double),
                ("alpha_k", ctypes.c_void_p), ("L", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("beta_v", ctypes.c_void_p)]


@pytest.mark.parametrize("K,V,beta,alpha,L,D,N", [
    (0, 10, 0.01, 0.1, 100, 1, 1),        # K < 1
    (5000, 10, 0.01, 0.1, 100, 1, 1),     # K > 4096
    (10, 0, 0.01, 0.1, 100, 1, 1),        # V < 1
    (4096, 600000, 0.01, 0.1, 100, 1, 1),  # K*V >= 2^31
    (1000, 1048576, 0.01, 0.1, 100, 1, 1),  # V * (K rounded up to 64) = 2^30
    (10, 10, 0.0, 0.1, 100, 1, 1),        # beta = 0
    (10, 10, 20.0, 0.1, 100, 1, 1),       # beta > 16 (zero-truncated tables would not saturate)
    (10, 10, 0.01, -1.0, 100, 1, 1),      # alpha < 0
    (10, 10, 0.01, 0.1, 0, 1, 1),         # L = 0
    (10, 10, 0.01, 0.1, 100, -1, 1),      # D < 0
])
def test_plan_create_rejects_bad_arguments(lib, K, V, beta, alpha, L, D, N):
    d = Desc(K, V, beta, alpha, None, L, 1)
    h = ctypes.c_void_p()
    st = lib.pulda_plan_create(ctypes.byref(d), ctypes.c_int64(D), ctypes.c_int64(N), ctypes.byref(h))
    assert st == -1 and not h.value
    lib.pulda_last_error.restype = ctypes.c_char_p
    assert lib.pulda_last_error()


def test_plan_create_per_word_priors(lib):
    import numpy as np
    good = np.full(10, 0.05)
    for bv, ok in [(good, True), (np.r_[good[:9], 0.0], False), (np.r_[good[:9], 17.0], False),
                   (np.r_[good[:9], np.nan], False)]:
        buf = np.ascontiguousarray(bv, dtype=np.float64)
        d = Desc(10, 10, 0.0, 0.1, None, 100, 1, buf.ctypes.data_as(ctypes.c_void_p))
        h = ctypes.c_void_p()
        st = lib.pulda_plan_create(ctypes.byref(d), ctypes.c_int64(1), ctypes.c_int64(1), ctypes.byref(h))
        assert (st == 0) == ok, bv
        if ok:
            lib.pulda_plan_destroy(h)


def test_plan_workspace_and_state_errors(lib):
    d = Desc(1000, 28000, 0.01, 0.1, None, 100, 1)
    h = ctypes.c_void_p()
    assert lib.pulda_plan_create(ctypes.byref(d), ctypes.c_int64(40000), ctypes.c_int64(6_500_000),
                                 ctypes.byref(h)) == 0
    nbytes = ctypes.c_int64()
    assert lib.pulda_plan_workspace_bytes(h, ctypes.byref(nbytes)) == 0
    # z, n, gamma, phi, CSC (u16 + f32 + u64), order ...: at least this much
    assert nbytes.value >= 6_500_000 * 2 + 1000 * 28000 * (4 * 3 + 14)
    # unbound: every state-changing call reports the state, not a crash
    assert lib.pulda_phi_step(h, ctypes.c_uint32(1), None) == -2
    assert lib.pulda_z_step(h, ctypes.c_uint32(1), None) == -2
    assert lib.pulda_corpus_upload(h, ctypes.c_void_p(8), ctypes.c_void_p(8), None) == -2
    # a workspace smaller than required is refused before any device call
    assert lib.pulda_plan_bind(h, ctypes.c_void_p(256), ctypes.c_int64(nbytes.value - 1)) == -4
    lib.pulda_plan_destroy(h)
