"""Python binding of libpulda.so (the C ABI in include/pulda.h).

Argument marshalling only: every step of the sampler runs in the library's
HIP kernels.  PyTorch provides device memory (the workspaces the library
carves its buffers from) and the stream.  There is no fallback: if the
compiled library is missing the import fails.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpulda.so")

PULDA_OK, ERR_INVALID_ARG, ERR_STATE, ERR_DEVICE, ERR_NO_MEMORY, ERR_CAPACITY, ERR_CORPUS = 0, -1, -2, -3, -4, -5, -6
# scratch of pulda_heldout_loglik_noalloc (PULDA_HELDOUT_NOALLOC_SCRATCH_BYTES in pulda.h)
HELDOUT_NOALLOC_SCRATCH_BYTES = 32 << 20


class PuldaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"pulda status {status}: {message}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
                          "or `python paper_1704_03581_amd/build.py`")
    return C.CDLL(LIB_PATH)


_lib = _load()
vp, i32, i64, u32, u64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double


class ModelDesc(C.Structure):
    _fields_ = [("K", i32), ("V", i32), ("beta", f64), ("alpha", f64), ("alpha_k", C.POINTER(f64)),
                ("L", i32), ("seed", u64), ("beta_v", C.POINTER(f64))]


class CountsView(C.Structure):
    _fields_ = [("n_colptr", vp), ("n_topic", vp), ("n_count", vp), ("nk", vp), ("m_rowptr", vp),
                ("m_topic", vp), ("m_count", vp)]


class PhiView(C.Structure):
    _fields_ = [("colptr", vp), ("topic", vp), ("gamma", vp), ("phi", vp), ("alias_thr", vp),
                ("alias_topic", vp), ("sigma_a", vp), ("S", vp)]


class SweepStats(C.Structure):
    _fields_ = [("degenerate_tokens", i64), ("sum_J", i64), ("sum_A", i64), ("z_steps", i64), ("nnz_phi", i64),
                ("empty_rows", i64), ("ms_phi", f64), ("ms_z", f64), ("ms_ll", f64), ("n_phi", i64), ("n_z", i64),
                ("n_ll", i64), ("sum_J_b", i64), ("fallback_draws", i64)]


class FoldinDesc(C.Structure):
    _fields_ = [("sweeps", i32), ("burn_in", i32), ("max_slots", i32), ("arena_tokens", i32), ("max_len", i32),
                ("group", i32), ("seed", u64)]


class FoldinResult(C.Structure):
    _fields_ = [("request_id", u32), ("kept", i32), ("dropped", i32), ("pad", i32), ("loglik", f64)]


_SIGS = {
    "pulda_plan_create": [C.POINTER(ModelDesc), i64, i64, C.POINTER(vp)],
    "pulda_plan_workspace_bytes": [vp, C.POINTER(i64)],
    "pulda_plan_bind": [vp, vp, i64],
    "pulda_corpus_upload": [vp, vp, vp, vp],
    "pulda_init": [vp, vp, vp],
    "pulda_set_z": [vp, vp, vp],
    "pulda_get_z": [vp, vp, vp],
    "pulda_set_counts": [vp, vp, vp],
    "pulda_phi_step": [vp, u32, vp],
    "pulda_z_step": [vp, u32, vp],
    "pulda_sweep": [vp, u32, i32, C.POINTER(f64), vp],
    "pulda_loglik": [vp, C.POINTER(f64), vp],
    "pulda_counts_sizes": [vp, C.POINTER(i64), C.POINTER(i64), vp],
    "pulda_counts": [vp, C.POINTER(CountsView), vp],
    "pulda_get_counts_dense": [vp, vp, vp, vp],
    "pulda_phi_nnz": [vp, C.POINTER(i64), vp],
    "pulda_get_phi": [vp, C.POINTER(PhiView), vp],
    "pulda_set_phi": [vp, C.POINTER(PhiView), vp],
    "pulda_stats": [vp, C.POINTER(SweepStats), vp],
    "pulda_set_schedule": [vp, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)],
    "pulda_get_schedule": [vp, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32),
                           C.POINTER(i32)],
    "pulda_autotune": [vp, u32, i32, vp],
    "pulda_set_graph": [vp, i32],
    "pulda_set_timing": [vp, i32],
    "pulda_set_fused_loglik": [vp, i32],
    "pulda_set_phi_method": [vp, i32],
    "pulda_heldout_workspace_bytes": [vp, i64, i64, i32, C.POINTER(i64)],
    "pulda_heldout_loglik": [vp, i64, vp, vp, vp, i32, i32, u64, vp, i64, vp, vp, vp, vp],
    "pulda_heldout_loglik_noalloc": [vp, i64, vp, vp, vp, i32, i32, u64, vp, vp, vp, vp],
    "pulda_get_gamma_dense": [vp, vp, vp, vp],
    "pulda_foldin_create": [vp, C.POINTER(FoldinDesc), C.POINTER(vp)],
    "pulda_foldin_workspace_bytes": [vp, C.POINTER(i64)],
    "pulda_foldin_bind": [vp, vp, i64],
    "pulda_foldin_submit": [vp, u32, vp, i32, vp],
    "pulda_foldin_step": [vp, i32, vp],
    "pulda_foldin_poll": [vp, C.POINTER(FoldinResult), vp, i32, C.POINTER(i32), vp],
    "pulda_foldin_poll_previous": [vp, C.POINTER(FoldinResult), vp, i32, C.POINTER(i32)],
    "pulda_foldin_occupancy": [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)],
    "pulda_foldin_run_one": [vp, u32, vp, i32, vp, C.POINTER(FoldinResult), vp],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = i32
_lib.pulda_last_error.restype = C.c_char_p
_lib.pulda_version.restype = C.c_char_p
_lib.pulda_plan_destroy.argtypes = [vp]
_lib.pulda_plan_destroy.restype = None
_lib.pulda_foldin_destroy.argtypes = [vp]
_lib.pulda_foldin_destroy.restype = None

EXPORTED = sorted(list(_SIGS) + ["pulda_last_error", "pulda_version", "pulda_plan_destroy", "pulda_foldin_destroy"])


def _check(status: int):
    if status != PULDA_OK:
        raise PuldaError(status, _lib.pulda_last_error().decode())


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev_tensor(x, dtype, device) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x)).to(device=device, dtype=dtype).contiguous()


def _u16_to_i16(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint16).view(np.int16)


def version() -> str:
    return _lib.pulda_version().decode()


class Plan:
    """A sampler over one corpus on one device (plan + bound workspace)."""

    def __init__(self, K: int, V: int, D: int, N: int, alpha=0.1, beta: float = 0.01, L: int = 100,
                 seed: int = 1, device="cuda"):
        self.K, self.V, self.D, self.N = K, V, D, N
        self.device = torch.device(device)
        # beta: the symmetric prior, or a vector of V per-word priors
        desc = ModelDesc(K=K, V=V, beta=float(np.mean(beta)) if np.ndim(beta) else float(beta),
                         alpha=float(np.mean(alpha)) if np.ndim(alpha) else float(alpha),
                         alpha_k=None, L=L, seed=seed, beta_v=None)
        self._alpha_buf = None
        if np.ndim(alpha):
            self._alpha_buf = np.ascontiguousarray(alpha, dtype=np.float64)
            desc.alpha_k = self._alpha_buf.ctypes.data_as(C.POINTER(f64))
        self._beta_buf = None
        if np.ndim(beta):
            self._beta_buf = np.ascontiguousarray(np.broadcast_to(beta, (V,)), dtype=np.float64)
            desc.beta_v = self._beta_buf.ctypes.data_as(C.POINTER(f64))
        self.alpha = np.broadcast_to(np.asarray(alpha, dtype=np.float64), (K,)).copy()
        self.beta, self.L, self.seed = beta, L, seed
        h = vp()
        _check(_lib.pulda_plan_create(C.byref(desc), D, N, C.byref(h)))
        self._h = h
        nbytes = i64()
        _check(_lib.pulda_plan_workspace_bytes(h, C.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_off = (-base) % 256
        with torch.cuda.device(self.device):
            _check(_lib.pulda_plan_bind(h, C.c_void_p(base + self._ws_off), nbytes.value))
        self._corpus = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.pulda_plan_destroy(h)
            self._h = None

    # corpus and state ------------------------------------------------------
    def upload(self, doc_off, words, stream=None):
        doc_off = _dev_tensor(doc_off, torch.int64, self.device)
        words = _dev_tensor(words, torch.int32, self.device)
        self._corpus = (doc_off, words)
        _check(_lib.pulda_corpus_upload(self._h, _ptr(doc_off), _ptr(words), _stream(stream)))

    def init(self, z0=None, stream=None):
        zt = None if z0 is None else _dev_tensor(_u16_to_i16(z0), torch.int16, self.device)
        _check(_lib.pulda_init(self._h, _ptr(zt), _stream(stream)))
        if zt is not None:
            torch.cuda.current_stream(self.device).synchronize()

    def set_z(self, z, stream=None):
        zt = _dev_tensor(_u16_to_i16(z), torch.int16, self.device)
        _check(_lib.pulda_set_z(self._h, _ptr(zt), _stream(stream)))
        torch.cuda.current_stream(self.device).synchronize()

    def get_z(self, stream=None) -> np.ndarray:
        zt = torch.empty(max(self.N, 1), dtype=torch.int16, device=self.device)
        _check(_lib.pulda_get_z(self._h, _ptr(zt), _stream(stream)))
        return zt[: self.N].cpu().numpy().view(np.uint16)

    def set_counts(self, n_word_major, stream=None):
        nt = _dev_tensor(n_word_major, torch.int32, self.device)
        _check(_lib.pulda_set_counts(self._h, _ptr(nt), _stream(stream)))
        torch.cuda.current_stream(self.device).synchronize()

    # Algorithm 2 -------------------------------------------------------------
    def phi_step(self, t: int, stream=None):
        _check(_lib.pulda_phi_step(self._h, t, _stream(stream)))

    def z_step(self, t: int, stream=None):
        _check(_lib.pulda_z_step(self._h, t, _stream(stream)))

    def sweep(self, t_first: int, n: int, want_ll: bool = True, stream=None):
        if want_ll:
            ll = (f64 * max(n, 1))()
            _check(_lib.pulda_sweep(self._h, t_first, n, ll, _stream(stream)))
            return np.array(ll[:n])
        _check(_lib.pulda_sweep(self._h, t_first, n, None, _stream(stream)))
        return None

    def loglik(self, stream=None) -> float:
        out = f64()
        _check(_lib.pulda_loglik(self._h, C.byref(out), _stream(stream)))
        return out.value

    # counts / Phi ------------------------------------------------------------
    def counts_dense(self, stream=None):
        """n as a (K, V) int32 array (the paper's orientation) and n_k."""
        n = torch.empty(self.V * self.K, dtype=torch.int32, device=self.device)
        nk = torch.empty(self.K, dtype=torch.int64, device=self.device)
        _check(_lib.pulda_get_counts_dense(self._h, _ptr(n), _ptr(nk), _stream(stream)))
        return n.view(self.V, self.K).t().contiguous().cpu().numpy(), nk.cpu().numpy()

    def counts(self, stream=None):
        nn, nm = i64(), i64()
        _check(_lib.pulda_counts_sizes(self._h, C.byref(nn), C.byref(nm), _stream(stream)))
        d = self.device
        out = dict(n_colptr=torch.empty(self.V + 1, dtype=torch.int64, device=d),
                   n_topic=torch.empty(max(nn.value, 1), dtype=torch.int16, device=d),
                   n_count=torch.empty(max(nn.value, 1), dtype=torch.int32, device=d),
                   nk=torch.empty(self.K, dtype=torch.int64, device=d),
                   m_rowptr=torch.empty(self.D + 1, dtype=torch.int64, device=d),
                   m_topic=torch.empty(max(nm.value, 1), dtype=torch.int16, device=d),
                   m_count=torch.empty(max(nm.value, 1), dtype=torch.int32, device=d))
        view = CountsView(*[C.c_void_p(out[k].data_ptr()) for k in
                            ["n_colptr", "n_topic", "n_count", "nk", "m_rowptr", "m_topic", "m_count"]])
        _check(_lib.pulda_counts(self._h, C.byref(view), _stream(stream)))
        res = {k: v.cpu().numpy() for k, v in out.items()}
        res["n_topic"] = res["n_topic"][: nn.value].view(np.uint16)
        res["n_count"] = res["n_count"][: nn.value]
        res["m_topic"] = res["m_topic"][: nm.value].view(np.uint16)
        res["m_count"] = res["m_count"][: nm.value]
        return res

    def phi_nnz(self, stream=None) -> int:
        n = i64()
        _check(_lib.pulda_phi_nnz(self._h, C.byref(n), _stream(stream)))
        return n.value

    def get_phi(self, stream=None) -> dict:
        nnz = self.phi_nnz(stream)
        d = self.device
        t = dict(colptr=torch.empty(self.V + 1, dtype=torch.int64, device=d),
                 topic=torch.empty(max(nnz, 1), dtype=torch.int16, device=d),
                 gamma=torch.empty(max(nnz, 1), dtype=torch.int32, device=d),
                 phi=torch.empty(max(nnz, 1), dtype=torch.float32, device=d),
                 alias_thr=torch.empty(max(nnz, 1), dtype=torch.int32, device=d),
                 alias_topic=torch.empty(max(nnz, 1), dtype=torch.int16, device=d),
                 sigma_a=torch.empty(self.V, dtype=torch.float64, device=d),
                 S=torch.empty(self.K, dtype=torch.int64, device=d))
        view = PhiView(*[C.c_void_p(t[k].data_ptr()) for k in
                         ["colptr", "topic", "gamma", "phi", "alias_thr", "alias_topic", "sigma_a", "S"]])
        _check(_lib.pulda_get_phi(self._h, C.byref(view), _stream(stream)))
        out = {k: v.cpu().numpy() for k, v in t.items()}
        for k in ("topic", "gamma", "phi", "alias_thr", "alias_topic"):
            out[k] = out[k][:nnz]
        out["topic"] = out["topic"].view(np.uint16)
        out["alias_topic"] = out["alias_topic"].view(np.uint16)
        out["alias_thr"] = out["alias_thr"].view(np.uint32)
        return out

    def set_phi(self, colptr, topic, phi, alias_thr, alias_topic, sigma_a, stream=None):
        d = self.device
        t = dict(colptr=_dev_tensor(colptr, torch.int64, d),
                 topic=_dev_tensor(_u16_to_i16(topic), torch.int16, d),
                 phi=_dev_tensor(phi, torch.float32, d),
                 alias_thr=_dev_tensor(np.ascontiguousarray(alias_thr, np.uint32).view(np.int32), torch.int32, d),
                 alias_topic=_dev_tensor(_u16_to_i16(alias_topic), torch.int16, d),
                 sigma_a=_dev_tensor(sigma_a, torch.float64, d))
        view = PhiView(_ptr(t["colptr"]), _ptr(t["topic"]), None, _ptr(t["phi"]), _ptr(t["alias_thr"]),
                       _ptr(t["alias_topic"]), _ptr(t["sigma_a"]), None)
        _check(_lib.pulda_set_phi(self._h, C.byref(view), _stream(stream)))
        torch.cuda.current_stream(self.device).synchronize()

    def stats(self, stream=None) -> dict:
        s = SweepStats()
        _check(_lib.pulda_stats(self._h, C.byref(s), _stream(stream)))
        return {k: getattr(s, k) for k, _ in SweepStats._fields_}

    # schedule ------------------------------------------------------------------
    def set_schedule(self, min_len, group, docs_per_item, side_ratio=None):
        nb = len(min_len)
        a = (i32 * nb)(*min_len)
        b = (i32 * nb)(*group)
        c = (i32 * nb)(*docs_per_item)
        d = None if side_ratio is None else (i32 * nb)(*side_ratio)
        _check(_lib.pulda_set_schedule(self._h, nb, a, b, c, d))

    def get_schedule(self):
        nb = i32()
        a, b, c, d = (i32 * 64)(), (i32 * 64)(), (i32 * 64)(), (i32 * 64)()
        _check(_lib.pulda_get_schedule(self._h, 64, C.byref(nb), a, b, c, d))
        n = nb.value
        return list(a[:n]), list(b[:n]), list(c[:n]), list(d[:n])

    def autotune(self, t: int, reps: int = 2, stream=None):
        _check(_lib.pulda_autotune(self._h, t, reps, _stream(stream)))
        return self.get_schedule()

    def set_graph(self, enable: bool):
        _check(_lib.pulda_set_graph(self._h, 1 if enable else 0))

    def heldout_loglik(self, docs, req=None, particles: int = 20, group: int = 32, seed: int = 1,
                       want_Z: bool = False, stream=None, noalloc: bool = False):
        """Left-to-right estimates of log p(w_d | Phi, alpha) for new
        documents (lists of word ids) against this plan's Phi.  req: request
        ids (default 0..D-1), the keys of the random numbers.  Returns
        (ll fp64[D], kept int32[D]) and, with want_Z, each document's
        Z (particles x kept) array.  noalloc: call the entry point that
        takes no workspace (the library's own scratch, of
        HELDOUT_NOALLOC_SCRATCH_BYTES)."""
        D = len(docs)
        lens = np.array([len(d) for d in docs], dtype=np.int64)
        off = np.zeros(D + 1, np.int64)
        np.cumsum(lens, out=off[1:])
        N = int(off[-1])
        words = np.concatenate([np.asarray(d, np.int32) for d in docs]) if N else np.zeros(1, np.int32)
        req = np.arange(D, dtype=np.uint32) if req is None else np.asarray(req, np.uint32)
        dv = self.device
        off_t = torch.from_numpy(off).to(dv)
        words_t = torch.from_numpy(words).to(dv)
        req_t = torch.from_numpy(np.ascontiguousarray(req).view(np.int32)).to(dv)
        ll = torch.empty(max(D, 1), dtype=torch.float64, device=dv)
        kept = torch.empty(max(D, 1), dtype=torch.int32, device=dv)
        Z = torch.empty(max(N * particles, 1), dtype=torch.float64, device=dv) if want_Z else None
        if noalloc:
            _check(_lib.pulda_heldout_loglik_noalloc(self._h, D, _ptr(off_t), _ptr(words_t), _ptr(req_t), particles,
                                                     group, seed, _ptr(ll), _ptr(kept), _ptr(Z) if want_Z else None,
                                                     _stream(stream)))
        else:
            nbytes = i64()
            _check(_lib.pulda_heldout_workspace_bytes(self._h, D, N, particles, C.byref(nbytes)))
            ws = torch.empty(max(nbytes.value, 1) + 256, dtype=torch.uint8, device=dv)
            base = (ws.data_ptr() + 255) // 256 * 256
            _check(_lib.pulda_heldout_loglik(self._h, D, _ptr(off_t), _ptr(words_t), _ptr(req_t), particles, group,
                                             seed, C.c_void_p(base), nbytes.value, _ptr(ll), _ptr(kept),
                                             _ptr(Z) if want_Z else None, _stream(stream)))
        ll_h = ll.cpu().numpy()[:D]
        kept_h = kept.cpu().numpy()[:D]
        if not want_Z:
            return ll_h, kept_h
        Zh = Z.cpu().numpy()
        Zs = [Zh[off[d] * particles: off[d] * particles + particles * lens[d]].reshape(particles, lens[d])[:, :kept_h[d]]
              for d in range(D)]
        return ll_h, kept_h, Zs

    PHI_METHODS = {"polya_urn": 0, "dirichlet": 1}

    def set_phi_method(self, method: str):
        """Phi-step of phi_step and sweep: "polya_urn" (Algorithm 2, the
        default) or "dirichlet" (Algorithm 1: Gamma draws)."""
        if method not in self.PHI_METHODS:
            raise ValueError(f"unknown Phi-step method {method!r}")
        _check(_lib.pulda_set_phi_method(self._h, self.PHI_METHODS[method]))

    def gamma_dense(self, stream=None):
        """After a Dirichlet Phi-step: the Gamma draws as a (K, V) fp64 array
        (the paper's orientation) and the row sums S (fp64)."""
        g = torch.empty(self.V * self.K, dtype=torch.float64, device=self.device)
        S = torch.empty(self.K, dtype=torch.float64, device=self.device)
        _check(_lib.pulda_get_gamma_dense(self._h, _ptr(g), _ptr(S), _stream(stream)))
        return g.view(self.V, self.K).t().contiguous().cpu().numpy(), S.cpu().numpy()

    def set_fused_loglik(self, enable: bool):
        _check(_lib.pulda_set_fused_loglik(self._h, 1 if enable else 0))

    def set_timing(self, enable: bool):
        _check(_lib.pulda_set_timing(self._h, 1 if enable else 0))


class FoldIn:
    """Fold-in server over a plan's Phi: continuous batching of requests."""

    def __init__(self, plan: Plan, sweeps: int = 50, burn_in: int = 25, max_slots: int = 4096,
                 arena_tokens: int = 4 << 20, max_len: int = 5000, group: int = 64, seed: int = 7):
        self.plan = plan
        self.K = plan.K
        desc = FoldinDesc(sweeps=sweeps, burn_in=burn_in, max_slots=max_slots, arena_tokens=arena_tokens,
                          max_len=max_len, group=group, seed=seed)
        self.desc = desc
        h = vp()
        _check(_lib.pulda_foldin_create(plan._h, C.byref(desc), C.byref(h)))
        self._h = h
        nbytes = i64()
        _check(_lib.pulda_foldin_workspace_bytes(h, C.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=plan.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        _check(_lib.pulda_foldin_bind(h, C.c_void_p(base + off), nbytes.value))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.pulda_foldin_destroy(h)
            self._h = None

    def submit(self, request_id: int, words, stream=None) -> bool:
        """True if admitted, False if the server is full right now."""
        w = np.ascontiguousarray(words, dtype=np.int32)
        st = _lib.pulda_foldin_submit(self._h, request_id, w.ctypes.data_as(vp), len(w), _stream(stream))
        if st == ERR_CAPACITY:
            return False
        _check(st)
        return True

    def step(self, draws: int, stream=None):
        """Advance every resident request by up to `draws` token draws."""
        _check(_lib.pulda_foldin_step(self._h, draws, _stream(stream)))

    def poll(self, cap: int = 4096, stream=None, previous: bool = False):
        """Finished requests.  previous: those finished by the step before the
        latest (pulda_foldin_poll_previous: the latest step keeps running)."""
        # result buffers are reused across polls
        if getattr(self, "_poll_cap", 0) < cap:
            self._poll_res = (FoldinResult * cap)()
            self._poll_theta = np.empty((cap, self.K), np.float32)
            self._poll_cap = cap
        res, theta = self._poll_res, self._poll_theta
        n = i32()
        if previous:
            _check(_lib.pulda_foldin_poll_previous(self._h, res, theta.ctypes.data_as(vp), cap, C.byref(n)))
        else:
            _check(_lib.pulda_foldin_poll(self._h, res, theta.ctypes.data_as(vp), cap, C.byref(n),
                                          _stream(stream)))
        out = []
        for j in range(n.value):
            r = res[j]
            out.append(dict(request_id=r.request_id, kept=r.kept, dropped=r.dropped, loglik=r.loglik,
                            theta=theta[j].copy()))
        return out

    def occupancy(self):
        a, b, c = i32(), i32(), i32()
        _check(_lib.pulda_foldin_occupancy(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return dict(resident=a.value, free_slots=b.value, free_tokens=c.value)

    def run_one(self, request_id: int, words, stream=None) -> dict:
        w = np.ascontiguousarray(words, dtype=np.int32)
        theta = np.zeros(self.K, np.float32)
        r = FoldinResult()
        _check(_lib.pulda_foldin_run_one(self._h, request_id, w.ctypes.data_as(vp), len(w),
                                         theta.ctypes.data_as(vp), C.byref(r), _stream(stream)))
        return dict(request_id=r.request_id, kept=r.kept, dropped=r.dropped, loglik=r.loglik, theta=theta)
