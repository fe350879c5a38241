"""SuCo on MI355X: Python binding of the C ABI in include/suco.h.

Argument marshalling only: tensors are checked for device, dtype and layout
and their data pointers are handed to libsuco.so; every step of the search
runs in the library's HIP kernels.  PyTorch provides device memory and the
current stream.  There is no fallback: if the compiled library is missing,
loading fails with an error that says how to build it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsuco.so")

SUCO_OK, SUCO_E_INVAL, SUCO_E_NOMEM, SUCO_E_HIP, SUCO_E_STATE, SUCO_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5

EXPORTED = (
    "suco_version", "suco_last_error", "suco_count_A", "suco_count_B", "suco_build",
    "suco_build_from_index", "suco_index_export", "suco_index_info", "suco_index_free", "suco_query",
    "suco_query_alpha", "suco_query_debug", "suco_collide_select", "suco_rerank", "suco_profile",
    "suco_profile_read", "suco_batcher_create", "suco_batcher_query", "suco_batcher_tuning",
    "suco_batcher_free", "suco_mlp_num_params", "suco_mlp_create", "suco_mlp_set_norm", "suco_mlp_get_params",
    "suco_mlp_set_params", "suco_mlp_forward_backward", "suco_mlp_train_epoch", "suco_mlp_predict",
    "suco_mlp_free", "suco_query_features", "suco_query_learned", "suco_batcher_set_model",
    "suco_query_bf16", "suco_query_bf16_debug", "suco_index_flags", "suco_index_save", "suco_index_load",
    "suco_query_noalloc", "suco_query_sclinear", "suco_index_set_activation", "suco_batcher_query_multi",
)

STAGES = ("activate", "collide", "select", "rerank", "merge", "centres_bf16", "rerank_bf16", "survivors", "order",
          "collide_sparse")


class SucoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"suco error {code}: {msg}")
        self.code = code


class BuildParams(C.Structure):
    _fields_ = [("iters", C.c_int32), ("seed", C.c_uint64), ("tile_max", C.c_int32),
                ("query_chunk", C.c_int32), ("flags", C.c_int32)]


BUILD_NO_BYTE_ROWS = 1
BUILD_BF16 = 2
BUILD_NO_SPARSE = 4
BUILD_L1 = 8
BF16_S1 = 1
INDEX_BYTE_ROWS, INDEX_BF16, INDEX_L1, INDEX_SPARSE = 1, 2, 4, 8
ACT_DYNAMIC, ACT_MULTISEQ = 0, 1


_lib = None
P = C.c_void_p
i64, i32, dbl = C.c_int64, C.c_int32, C.c_double


def lib():
    """Load libsuco.so (built by __graft_entry__.build() or paper_2411_14754_amd._build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        L.suco_version.restype = C.c_int
        L.suco_last_error.restype = C.c_char_p
        L.suco_count_A.restype = i64
        L.suco_count_A.argtypes = [dbl, i64]
        L.suco_count_B.restype = i64
        L.suco_count_B.argtypes = [dbl, i64, i32]
        L.suco_build.argtypes = [P, i64, i32, i32, i32, C.POINTER(BuildParams), P, C.POINTER(P)]
        L.suco_build_from_index.argtypes = [P, i64, i32, i32, i32, P, P, C.POINTER(BuildParams), P,
                                            C.POINTER(P)]
        L.suco_index_export.argtypes = [P, P, P]
        L.suco_index_info.argtypes = [P, P, P, P, P]
        L.suco_index_free.argtypes = [P]
        L.suco_index_flags.argtypes = [P, P]
        L.suco_index_set_activation.argtypes = [P, i32]
        L.suco_index_save.argtypes = [P, C.c_char_p]
        L.suco_index_load.argtypes = [C.c_char_p, C.POINTER(BuildParams), P, C.POINTER(P)]
        L.suco_query.argtypes = [P, P, i64, i32, dbl, dbl, P, P, P]
        L.suco_query_alpha.argtypes = [P, P, i64, i32, P, dbl, P, P, P]
        L.suco_query_noalloc.argtypes = [P, P, i64, i32, dbl, dbl, P, P, P]
        L.suco_query_sclinear.argtypes = [P, P, i64, i32, dbl, dbl, P, P, P, P]
        L.suco_query_debug.argtypes = [P, P, i64, i32, P, dbl, dbl, P, P, P, P, P, P, P, P, P]
        L.suco_collide_select.argtypes = [P, i64, P, P, i32, dbl, P, P, P]
        L.suco_rerank.argtypes = [P, P, i64, P, i64, i32, P, P, P]
        L.suco_profile.argtypes = [P, C.c_int]
        L.suco_profile_read.argtypes = [P, P, P]
        L.suco_batcher_create.argtypes = [P, i32, i32, dbl, C.c_char_p, C.POINTER(P)]
        L.suco_batcher_query.argtypes = [P, P, i64, P, dbl, P, P, P]
        L.suco_batcher_query_multi.argtypes = [P, i32, P, P, P, dbl, P, P, P]
        L.suco_batcher_tuning.argtypes = [P, i32, P, P]
        L.suco_batcher_free.argtypes = [P]
        L.suco_mlp_num_params.restype = i64
        L.suco_mlp_num_params.argtypes = [i32, i32]
        L.suco_mlp_create.argtypes = [i32, i32, P, C.c_uint64, C.POINTER(P)]
        L.suco_mlp_set_norm.argtypes = [P, P, P]
        L.suco_mlp_get_params.argtypes = [P, P]
        L.suco_mlp_set_params.argtypes = [P, P]
        L.suco_mlp_forward_backward.argtypes = [P, P, P, i64, P, P, P]
        L.suco_mlp_train_epoch.argtypes = [P, P, P, i64, i32, C.c_float, P, P, P]
        L.suco_mlp_predict.argtypes = [P, P, i64, C.c_float, C.c_float, C.c_float, P, P, P]
        L.suco_mlp_free.argtypes = [P]
        L.suco_query_features.argtypes = [P, P, i64, P, P]
        L.suco_query_learned.argtypes = [P, P, P, i64, i32, dbl, C.c_float, C.c_float, C.c_float, P, P, P, P]
        L.suco_batcher_set_model.argtypes = [P, P, C.c_float, C.c_float, C.c_float]
        L.suco_query_bf16.argtypes = [P, P, i64, i32, dbl, dbl, i32, P, P, P, P, P, P]
        L.suco_query_bf16_debug.argtypes = [P, P, i64, i32, dbl, dbl, i32, P, P, P, P, P, P, P, P, P, P, P]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != SUCO_OK:
        raise SucoError(rc, lib().suco_last_error().decode(errors="replace"))


def count_A(alpha: float, n: int) -> int:
    return int(lib().suco_count_A(float(alpha), int(n)))


def count_B(beta: float, n: int, k: int) -> int:
    return int(lib().suco_count_B(float(beta), int(n), int(k)))


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(t, dtype, shape=None, name="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def _opt(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Index:
    """A SuCo index resident on one GPU (Create Index, Alg. 2)."""

    def __init__(self, handle: int, n: int, d: int, ns: int, sqrt_k: int):
        self._h = C.c_void_p(handle)
        self.n, self.d, self.ns, self.sqrt_k = n, d, ns, sqrt_k
        self.K = sqrt_k * sqrt_k

    @staticmethod
    def _params(iters, seed, tile_max, query_chunk, flags=0):
        return BuildParams(iters, seed, tile_max, query_chunk, flags)

    @classmethod
    def build(cls, X, n_s: int, sqrt_k: int, iters: int = 25, seed: int = 1, tile_max: int = 0,
              query_chunk: int = 0, flags: int = 0, stream=None) -> "Index":
        torch = _torch()
        n, d = X.shape
        px = _dev(X, torch.float32, name="X")
        prm = cls._params(iters, seed, tile_max, query_chunk, flags)
        h = C.c_void_p()
        _check(lib().suco_build(px, n, d, n_s, sqrt_k, C.byref(prm), _stream(stream), C.byref(h)))
        return cls(h.value, n, d, n_s, sqrt_k)

    @classmethod
    def from_index(cls, X, n_s: int, sqrt_k: int, centroids: np.ndarray, assign: np.ndarray,
                   tile_max: int = 0, query_chunk: int = 0, flags: int = 0, stream=None) -> "Index":
        torch = _torch()
        n, d = X.shape
        px = _dev(X, torch.float32, name="X")
        cent = np.ascontiguousarray(centroids, np.float32).reshape(-1)
        asg = np.ascontiguousarray(assign, np.int32).reshape(-1)
        if cent.size != sqrt_k * d or asg.size != 2 * n_s * n:
            raise ValueError("centroids must hold sqrt_k*d values and assign 2*n_s*n values")
        prm = cls._params(0, 0, tile_max, query_chunk, flags)
        h = C.c_void_p()
        _check(lib().suco_build_from_index(px, n, d, n_s, sqrt_k, cent.ctypes.data_as(P),
                                           asg.ctypes.data_as(P), C.byref(prm), _stream(stream), C.byref(h)))
        return cls(h.value, n, d, n_s, sqrt_k)

    def save(self, path: str):
        """Write the index and its data to `path` (see suco_index_save)."""
        _check(lib().suco_index_save(self._h, os.fsencode(path)))

    @classmethod
    def load(cls, path: str, tile_max=None, query_chunk=None, flags=None, stream=None) -> "Index":
        """Read an index saved by save(); keyword arguments override the stored build parameters."""
        h = C.c_void_p()
        prm = None
        if tile_max is not None or query_chunk is not None or flags is not None:
            prm = C.byref(cls._params(0, 0, tile_max or 0, query_chunk or 0, flags or 0))
        _check(lib().suco_index_load(os.fsencode(path), prm, _stream(stream), C.byref(h)))
        n, d, ns, sk = i64(), i32(), i32(), i32()
        _check(lib().suco_index_info(h, C.byref(n), C.byref(d), C.byref(ns), C.byref(sk)))
        return cls(h.value, n.value, d.value, ns.value, sk.value)

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().suco_index_free(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            if _lib is not None and getattr(self, "_h", None) is not None and self._h.value:
                _lib.suco_index_free(self._h)
        except Exception:
            pass

    def profile(self, enable: bool = True):
        """Bracket every launch with HIP events on the query stream (see suco_profile)."""
        _check(lib().suco_profile(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        """{step: (total ms, launches)} since the last read (waits for the recorded work)."""
        ms = np.zeros(len(STAGES), np.float64)
        cnt = np.zeros(len(STAGES), np.int64)
        _check(lib().suco_profile_read(self._h, ms.ctypes.data_as(P), cnt.ctypes.data_as(P)))
        return {s: (float(ms[j]), int(cnt[j])) for j, s in enumerate(STAGES)}

    def flags(self) -> int:
        """INDEX_BYTE_ROWS | INDEX_BF16 | INDEX_L1 | INDEX_SPARSE bits (see suco_index_flags)."""
        f = C.c_int32(0)
        _check(lib().suco_index_flags(self._h, C.byref(f)))
        return int(f.value)

    def set_activation(self, form: int):
        """ACT_DYNAMIC (Alg. 3) or ACT_MULTISEQ for the queries that follow (see suco_index_set_activation)."""
        _check(lib().suco_index_set_activation(self._h, int(form)))

    def export(self):
        cent = np.zeros(self.sqrt_k * self.d, np.float32)
        asg = np.zeros((2 * self.ns, self.n), np.int32)
        _check(lib().suco_index_export(self._h, cent.ctypes.data_as(P), asg.ctypes.data_as(P)))
        return cent, asg

    def _out(self, nq, k):
        torch = _torch()
        return (torch.empty((nq, k), dtype=torch.int32, device="cuda"),
                torch.empty((nq, k), dtype=torch.float32, device="cuda"))

    def query(self, Q, k: int, alpha: float, beta: float, out=None, stream=None):
        """k-ANN Query (Alg. 4): returns (ids int32 [nq,k], dists float32 [nq,k])."""
        torch = _torch()
        nq = Q.shape[0]
        pq = _dev(Q, torch.float32, (nq, self.d), "Q")
        ids, dists = out if out is not None else self._out(nq, k)
        _check(lib().suco_query(self._h, pq, nq, k, float(alpha), float(beta), _dev(ids, torch.int32),
                                _dev(dists, torch.float32), _stream(stream)))
        return ids, dists

    def query_noalloc(self, Q, k: int, alpha: float, beta: float, out=None, stream=None):
        """suco_query with the library's fixed scratch as workspace (see suco_query_noalloc)."""
        torch = _torch()
        nq = Q.shape[0]
        pq = _dev(Q, torch.float32, (nq, self.d), "Q")
        ids, dists = out if out is not None else self._out(nq, k)
        _check(lib().suco_query_noalloc(self._h, pq, nq, k, float(alpha), float(beta), _dev(ids, torch.int32),
                                        _dev(dists, torch.float32), _stream(stream)))
        return ids, dists

    def query_sclinear(self, Q, k: int, alpha: float, beta: float, scores=False, out=None, stream=None):
        """SC-Linear (Alg. 1, see suco_query_sclinear): (ids, dists, scores uint8 [nq,n] or None)."""
        torch = _torch()
        nq = Q.shape[0]
        pq = _dev(Q, torch.float32, (nq, self.d), "Q")
        ids, dists = out if out is not None else self._out(nq, k)
        sc = torch.empty((nq, self.n), dtype=torch.uint8, device="cuda") if scores else None
        _check(lib().suco_query_sclinear(self._h, pq, nq, k, float(alpha), float(beta), _dev(ids, torch.int32),
                                         _dev(dists, torch.float32), _opt(sc), _stream(stream)))
        return ids, dists, sc

    def query_alpha(self, Q, k: int, alpha_q, beta: float, out=None, stream=None):
        torch = _torch()
        nq = Q.shape[0]
        pq = _dev(Q, torch.float32, (nq, self.d), "Q")
        pa = _dev(alpha_q, torch.float32, (nq,), "alpha_q")
        ids, dists = out if out is not None else self._out(nq, k)
        _check(lib().suco_query_alpha(self._h, pq, nq, k, pa, float(beta), _dev(ids, torch.int32),
                                      _dev(dists, torch.float32), _stream(stream)))
        return ids, dists

    def query_debug(self, Q, k: int, alpha: float, beta: float, alpha_q=None, stream=None,
                    scores=True, cand=True, cells=True, feat=True):
        """Alg. 4 with every intermediate exported (see suco_query_debug)."""
        torch = _torch()
        nq = Q.shape[0]
        B = count_B(beta, self.n, k)
        dev = "cuda"
        ids, dists = self._out(nq, k)
        o = dict(ids=ids, dists=dists)
        o["scores"] = torch.empty((nq, self.n), dtype=torch.uint8, device=dev) if scores else None
        o["cand"] = torch.empty((nq, B), dtype=torch.int32, device=dev) if cand else None
        o["ncells"] = torch.empty((nq, self.ns), dtype=torch.int32, device=dev)
        o["aprime"] = torch.empty((nq, self.ns), dtype=torch.int32, device=dev)
        o["cells"] = torch.empty((nq, self.ns, self.K), dtype=torch.uint16, device=dev) if cells else None
        o["feat"] = torch.empty((nq, 2 * self.ns), dtype=torch.float32, device=dev) if feat else None
        pa = _dev(alpha_q, torch.float32, (nq,), "alpha_q") if alpha_q is not None else None
        _check(lib().suco_query_debug(self._h, _dev(Q, torch.float32, (nq, self.d), "Q"), nq, k, pa,
                                      float(alpha), float(beta), _opt(ids), _opt(dists), _opt(o["scores"]),
                                      _opt(o["cand"]), _opt(o["ncells"]), _opt(o["aprime"]), _opt(o["cells"]),
                                      _opt(o["feat"]), _stream(stream)))
        return o

    def query_bf16(self, Q, k: int, alpha: float, beta: float, s1_bf16: bool = False, nsurv=True,
                   relerr=True, cdist=False, debug=False, out=None, stream=None):
        """BF16 split-precision query (see suco_query_bf16): returns a dict with ids, dists and
        the requested extras (nsurv int32 [nq], relerr float64 [nq,k], cdist float32
        [nq,2ns,sqrt_k]); debug=True adds scores, cand, ncells, aprime and cells as in query_debug."""
        torch = _torch()
        nq = Q.shape[0]
        pq = _dev(Q, torch.float32, (nq, self.d), "Q")
        ids, dists = out if out is not None else self._out(nq, k)
        dev = "cuda"
        o = dict(ids=ids, dists=dists)
        o["nsurv"] = torch.empty((nq,), dtype=torch.int32, device=dev) if nsurv else None
        o["relerr"] = torch.empty((nq, k), dtype=torch.float64, device=dev) if relerr else None
        o["cdist"] = (torch.empty((nq, 2 * self.ns, self.sqrt_k), dtype=torch.float32, device=dev)
                      if cdist else None)
        flags = BF16_S1 if s1_bf16 else 0
        head = (self._h, pq, nq, k, float(alpha), float(beta), flags, _dev(ids, torch.int32),
                _dev(dists, torch.float32), _opt(o["nsurv"]), _opt(o["relerr"]), _opt(o["cdist"]))
        if not debug:
            _check(lib().suco_query_bf16(*head, _stream(stream)))
            return o
        B = count_B(beta, self.n, k)
        o["scores"] = torch.empty((nq, self.n), dtype=torch.uint8, device=dev)
        o["cand"] = torch.empty((nq, B), dtype=torch.int32, device=dev)
        o["ncells"] = torch.empty((nq, self.ns), dtype=torch.int32, device=dev)
        o["aprime"] = torch.empty((nq, self.ns), dtype=torch.int32, device=dev)
        o["cells"] = torch.empty((nq, self.ns, self.K), dtype=torch.uint16, device=dev)
        _check(lib().suco_query_bf16_debug(*head, _opt(o["scores"]), _opt(o["cand"]), _opt(o["ncells"]),
                                           _opt(o["aprime"]), _opt(o["cells"]), _stream(stream)))
        return o

    def collide_select(self, cells, ncells, k: int, beta: float, want_scores=True, stream=None):
        """Steps 3-4 from given activated cells: returns (cand int32 [nq,B], scores uint8 [nq,n])."""
        torch = _torch()
        nq = cells.shape[0]
        B = count_B(beta, self.n, k)
        pc = _dev(cells, torch.uint16, (nq, self.ns, self.K), "cells")
        pn = _dev(ncells, torch.int32, (nq, self.ns), "ncells")
        cand = torch.empty((nq, B), dtype=torch.int32, device="cuda")
        sc = torch.empty((nq, self.n), dtype=torch.uint8, device="cuda") if want_scores else None
        _check(lib().suco_collide_select(self._h, nq, pc, pn, k, float(beta), _opt(sc), _dev(cand, torch.int32),
                                         _stream(stream)))
        return cand, sc

    def rerank(self, Q, cand, k: int, stream=None):
        """Step 5 on given candidates: returns (ids, dists)."""
        torch = _torch()
        nq, B = cand.shape
        pq = _dev(Q, torch.float32, (nq, self.d), "Q")
        ids, dists = self._out(nq, k)
        _check(lib().suco_rerank(self._h, pq, nq, _dev(cand, torch.int32), B, k, _dev(ids, torch.int32),
                                 _dev(dists, torch.float32), _stream(stream)))
        return ids, dists


class Batcher:
    """Batched query executor over an Index (see suco_batcher_create): one HIP
    graph per power-of-two batch-size bucket, tuned on first use."""

    def __init__(self, index: Index, max_batch: int, k: int, beta: float, tune_file: str | None = None):
        self.index, self.k, self.beta = index, k, beta
        h = C.c_void_p()
        _check(lib().suco_batcher_create(index._h, int(max_batch), int(k), float(beta),
                                         tune_file.encode() if tune_file else None, C.byref(h)))
        self._h = h

    def query(self, Q, alpha: float = 0.0, alpha_q=None, out=None, stream=None):
        torch = _torch()
        nq = Q.shape[0]
        pq = _dev(Q, torch.float32, (nq, self.index.d), "Q")
        pa = _dev(alpha_q, torch.float32, (nq,), "alpha_q") if alpha_q is not None else None
        ids, dists = out if out is not None else self.index._out(nq, self.k)
        _check(lib().suco_batcher_query(self._h, pq, nq, pa, float(alpha), _dev(ids, torch.int32),
                                        _dev(dists, torch.float32), _stream(stream)))
        return ids, dists

    def query_multi(self, Qs, alpha: float = 0.0, alpha_qs=None, outs=None, stream=None):
        """Several batches (up to 16) in one launch (suco_batcher_query_multi);
        returns [(ids, dists)] per batch."""
        torch = _torch()
        nb = len(Qs)
        if outs is None:
            outs = [self.index._out(q.shape[0], self.k) for q in Qs]
        PA = C.c_void_p * max(1, nb)
        pq, pa, pi, pd = PA(), PA(), PA(), PA()
        nq = (C.c_int64 * max(1, nb))()
        for j, Q in enumerate(Qs):
            n = Q.shape[0]
            nq[j] = n
            if n == 0:
                continue
            pq[j] = _dev(Q, torch.float32, (n, self.index.d), "Q")
            if alpha_qs is not None:
                pa[j] = _dev(alpha_qs[j], torch.float32, (n,), "alpha_q")
            pi[j] = _dev(outs[j][0], torch.int32, (n, self.k), "ids")
            pd[j] = _dev(outs[j][1], torch.float32, (n, self.k), "dists")
        _check(lib().suco_batcher_query_multi(self._h, nb, pq, nq, pa if alpha_qs is not None else None,
                                              float(alpha), pi, pd, _stream(stream)))
        return outs

    def set_model(self, mlp, scale: float = 1.0, alpha_min: float = 1e-4, alpha_max: float = 1.0):
        """Compute each batch's alphas with `mlp` inside the graph (None detaches)."""
        self._model = mlp
        _check(lib().suco_batcher_set_model(self._h, mlp._h if mlp is not None else None, float(scale),
                                            float(alpha_min), float(alpha_max)))

    def tuning(self, bucket: int):
        prm = np.zeros(3, np.int32)
        ms = C.c_double()
        _check(lib().suco_batcher_tuning(self._h, int(bucket), prm.ctypes.data_as(P), C.byref(ms)))
        return {"rows_per_part": int(prm[0]), "collide_grid_cap": int(prm[1]), "rerank_grid_cap": int(prm[2]),
                "ms": ms.value}

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().suco_batcher_free(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            if _lib is not None and getattr(self, "_h", None) is not None and self._h.value:
                _lib.suco_batcher_free(self._h)
        except Exception:
            pass


class MLP:
    """The learned activation-budget network (see suco_mlp_create)."""

    HIDDEN = 128

    def __init__(self, n_in: int, params: np.ndarray | None = None, seed: int = 1):
        self.n_in = n_in
        self.num_params = int(lib().suco_mlp_num_params(n_in, self.HIDDEN))
        if self.num_params < 0:
            raise ValueError("unsupported network shape")
        h = C.c_void_p()
        pp = None
        if params is not None:
            params = np.ascontiguousarray(params, np.float32).reshape(-1)
            if params.size != self.num_params:
                raise ValueError(f"expected {self.num_params} parameters")
            pp = params.ctypes.data_as(P)
        _check(lib().suco_mlp_create(n_in, self.HIDDEN, pp, C.c_uint64(seed), C.byref(h)))
        self._h = h

    def set_norm(self, mu, sigma):
        mu = np.ascontiguousarray(mu, np.float32)
        sigma = np.ascontiguousarray(sigma, np.float32)
        _check(lib().suco_mlp_set_norm(self._h, mu.ctypes.data_as(P), sigma.ctypes.data_as(P)))
        self.mu, self.sigma = mu, sigma

    def params(self) -> np.ndarray:
        out = np.zeros(self.num_params, np.float32)
        _check(lib().suco_mlp_get_params(self._h, out.ctypes.data_as(P)))
        return out

    def set_params(self, params):
        params = np.ascontiguousarray(params, np.float32).reshape(-1)
        _check(lib().suco_mlp_set_params(self._h, params.ctypes.data_as(P)))

    def forward_backward(self, F, t, stream=None):
        """(loss, gradient) on the GPU in FP32 for rows F [m, n_in] and targets t [m]."""
        torch = _torch()
        m = F.shape[0]
        g = torch.empty(self.num_params, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(lib().suco_mlp_forward_backward(self._h, _dev(F, torch.float32, (m, self.n_in), "F"),
                                               _dev(t, torch.float32, (m,), "t"), m, _opt(loss), _opt(g),
                                               _stream(stream)))
        return loss, g

    def train_epoch(self, F, t, batch: int, lr: float, order=None, want_loss=True, stream=None) -> float:
        torch = _torch()
        m = F.shape[0]
        po = _dev(order, torch.int32, (m,), "order") if order is not None else None
        ml = C.c_float(0.0)
        _check(lib().suco_mlp_train_epoch(self._h, _dev(F, torch.float32, (m, self.n_in), "F"),
                                          _dev(t, torch.float32, (m,), "t"), m, int(batch), float(lr), po,
                                          C.byref(ml) if want_loss else None, _stream(stream)))
        return float(ml.value)

    def predict(self, F, scale: float = 1.0, alpha_min: float = 1e-4, alpha_max: float = 1.0, stream=None):
        """BF16 inference: (y = predicted log alpha, alpha)."""
        torch = _torch()
        m = F.shape[0]
        y = torch.empty(m, dtype=torch.float32, device="cuda")
        a = torch.empty(m, dtype=torch.float32, device="cuda")
        _check(lib().suco_mlp_predict(self._h, _dev(F, torch.float32, (m, self.n_in), "F"), m, float(scale),
                                      float(alpha_min), float(alpha_max), _opt(y), _opt(a), _stream(stream)))
        return y, a

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().suco_mlp_free(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            if _lib is not None and getattr(self, "_h", None) is not None and self._h.value:
                _lib.suco_mlp_free(self._h)
        except Exception:
            pass


def query_features(index: Index, Q, stream=None):
    torch = _torch()
    nq = Q.shape[0]
    F = torch.empty((nq, 2 * index.ns + 1), dtype=torch.float32, device="cuda")
    _check(lib().suco_query_features(index._h, _dev(Q, torch.float32, (nq, index.d), "Q"), nq, _opt(F),
                                     _stream(stream)))
    return F


def query_learned(index: Index, mlp: MLP, Q, k: int, beta: float, scale: float, alpha_min: float = 1e-4,
                  alpha_max: float = 1.0, out=None, stream=None):
    """k-ANN query with per-query alphas from `mlp`: returns (ids, dists, alpha_used)."""
    torch = _torch()
    nq = Q.shape[0]
    ids, dists = out if out is not None else index._out(nq, k)
    au = torch.empty(nq, dtype=torch.float32, device="cuda")
    _check(lib().suco_query_learned(index._h, mlp._h, _dev(Q, torch.float32, (nq, index.d), "Q"), nq, k,
                                    float(beta), float(scale), float(alpha_min), float(alpha_max),
                                    _dev(ids, torch.int32), _dev(dists, torch.float32), _opt(au), _stream(stream)))
    return ids, dists, au
