"""SuCo FP64 oracle -- TEST INFRASTRUCTURE ONLY.

Plain CPU implementation of what the SuCo query path computes, used as the
parity judge for the GPU library and as the timed CPU baseline.  Only tests,
the smoke check and the benchmark's CPU-baseline leg may import it; the GPU
product path never does.  It shares no code with the GPU library.

The compiled part is ``suco_oracle.c`` (FP64 C, built by ``build()`` with gcc);
this module wraps it with ctypes and adds the FP64 NumPy pieces: the learned-
budget MLP (forward, analytic backward, Adam) and the BF16 rounding model.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "suco_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

P = C.c_void_p
i64 = C.c_int64
i32 = C.c_int


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP contraction off, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
                               "-fvisibility=hidden", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        L.so_count_A.restype = i64
        L.so_count_A.argtypes = [C.c_double, i64]
        L.so_count_B.restype = i64
        L.so_count_B.argtypes = [C.c_double, i64, i32]
        L.so_layout.argtypes = [i32, i32, P, P]
        L.so_init_ids.argtypes = [P, i64, i32, i32, i32, i32, C.c_uint64, i32, P]
        L.so_kmeans.argtypes = [P, i64, i32, i32, i32, i32, i32, P, P, P, P, i32]
        L.so_kmedians.argtypes = [P, i64, i32, i32, i32, i32, i32, P, P, P, P, i32]
        L.so_build_metric.argtypes = [P, i64, i32, i32, i32, i32, C.c_uint64, i32, P, P, P, P, i32]
        L.so_build.argtypes = [P, i64, i32, i32, i32, i32, C.c_uint64, P, P, P, P, i32]
        L.so_index_create.restype = P
        L.so_index_create.argtypes = [P, i64, i32, i32, i32, P, P]
        L.so_index_free.argtypes = [P]
        L.so_index_offs.restype = C.POINTER(C.c_int64)
        L.so_index_offs.argtypes = [P]
        L.so_index_ids.restype = C.POINTER(C.c_int32)
        L.so_index_ids.argtypes = [P]
        L.so_centroid_dists.argtypes = [P, P, i32, P]
        L.so_argsort.argtypes = [P, i32, P]
        L.so_da.restype = i64
        L.so_da.argtypes = [P, i32, P, P, P, P, i64, i32, P, P]
        L.so_da_trace.restype = i64
        L.so_da_trace.argtypes = [P, i32, P, P, P, P, i64, P, P, P]
        L.so_select.argtypes = [P, i64, i64, P]
        L.so_rerank.argtypes = [P, i32, P, P, i64, i32, P, P]
        L.so_rerank_metric.argtypes = [P, i32, P, P, i64, i32, i32, P, P]
        L.so_query.argtypes = [P, P, i64, i32, P, C.c_double, i32, P, P, P, P, P, P, i32]
        L.so_query_cells.restype = i64
        L.so_query_cells.argtypes = [P, P, i32, C.c_double, i32, P, P, P, P, P, P]
        L.so_sclinear_metric.argtypes = [P, i64, i32, i32, P, i64, i32, C.c_double, C.c_double, i32, P, P, P, i32]
        L.so_bruteforce.argtypes = [P, i64, i32, P, i64, i32, P, P, i32]
        L.so_bruteforce_metric.argtypes = [P, i64, i32, P, i64, i32, i32, P, P, i32]
        L.so_bf16.restype = C.c_double
        L.so_bf16.argtypes = [C.c_float]
        L.so_bf16_round.argtypes = [P, i64, P]
        L.so_index_set_s1_bf16.argtypes = [P, i32]
        L.so_index_set_metric.argtypes = [P, i32]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def count_A(alpha: float, n: int) -> int:
    return int(lib().so_count_A(float(alpha), int(n)))


def count_B(beta: float, n: int, k: int) -> int:
    return int(lib().so_count_B(float(beta), int(n), int(k)))


def layout(d: int, ns: int):
    dim0 = np.zeros(2 * ns, np.int32)
    w = np.zeros(2 * ns, np.int32)
    lib().so_layout(d, ns, _p(dim0), _p(w))
    return dim0, w


def init_ids(X: np.ndarray, ns: int, sk: int, seed: int, g: int) -> np.ndarray:
    X = np.ascontiguousarray(X, np.float32)
    n, d = X.shape
    dim0, w = layout(d, ns)
    out = np.zeros(sk, np.int64)
    lib().so_init_ids(_p(X), n, d, int(dim0[g]), int(w[g]), sk, C.c_uint64(seed), g, _p(out))
    return out


def kmeans(X, dim0, w, sk, iters, init, nthreads=None, metric=0):
    """Lloyd's k-means on one half (metric 0), or k-medians under L1 (metric 1, SuCo-L1)."""
    X = np.ascontiguousarray(X, np.float32)
    n, d = X.shape
    cent = np.zeros((sk, w), np.float64)
    assign = np.zeros(n, np.int32)
    obj = np.zeros(iters + 1, np.float64)
    init = np.ascontiguousarray(init, np.int64)
    fn = lib().so_kmedians if metric else lib().so_kmeans
    rc = fn(_p(X), n, d, dim0, w, sk, iters, _p(init), _p(cent), _p(assign), _p(obj),
            nthreads or default_threads())
    assert rc == 0
    return cent, assign, obj


def build_index(X: np.ndarray, ns: int, sk: int, iters: int = 25, seed: int = 1, nthreads=None, metric=0):
    """Alg. 2: returns (cent64 [sk*d], cent32 [sk*d], assign int32 [2ns][n], obj [2ns][iters+1]).
    metric 1 (SuCo-L1) clusters with k-medians under L1."""
    X = np.ascontiguousarray(X, np.float32)
    n, d = X.shape
    c64 = np.zeros(sk * d, np.float64)
    c32 = np.zeros(sk * d, np.float32)
    asg = np.zeros((2 * ns, n), np.int32)
    obj = np.zeros((2 * ns, iters + 1), np.float64)
    rc = lib().so_build_metric(_p(X), n, d, ns, sk, iters, C.c_uint64(seed), int(metric), _p(c64), _p(c32),
                               _p(asg), _p(obj), nthreads or default_threads())
    assert rc == 0
    return c64, c32, asg, obj


class Index:
    """The oracle's index over X with given FP32 centres and assignments."""

    def __init__(self, X, ns, sk, cent32, assign, metric=0):
        self.metric = int(metric)
        self.X = np.ascontiguousarray(X, np.float32)
        self.n, self.d = self.X.shape
        self.ns, self.sk, self.K = ns, sk, sk * sk
        self.cent32 = np.ascontiguousarray(cent32, np.float32).reshape(-1)
        self.assign = np.ascontiguousarray(assign, np.int32).reshape(2 * ns, self.n)
        self.h = lib().so_index_create(_p(self.X), self.n, self.d, ns, sk, _p(self.cent32), _p(self.assign))
        if not self.h:
            raise MemoryError("oracle index")
        lib().so_index_set_metric(self.h, self.metric)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.so_index_free(self.h)
            self.h = None

    def set_s1_bf16(self, on: bool = True):
        """Centre distances from BF16-rounded query halves and centres (the split-precision model)."""
        lib().so_index_set_s1_bf16(self.h, 1 if on else 0)

    def offs(self) -> np.ndarray:
        p = lib().so_index_offs(self.h)
        return np.ctypeslib.as_array(p, shape=(self.ns * (self.K + 1),)).reshape(self.ns, self.K + 1).copy()

    def ids(self) -> np.ndarray:
        p = lib().so_index_ids(self.h)
        return np.ctypeslib.as_array(p, shape=(self.ns * self.n,)).reshape(self.ns, self.n).copy()

    def centroid_dists(self, q, g):
        q = np.ascontiguousarray(q, np.float32)
        out = np.zeros(self.sk, np.float64)
        lib().so_centroid_dists(self.h, _p(q), g, _p(out))
        return out

    def cells(self, q, i, alpha, form=0):
        """Activated cells (retrieval order), A', and the sorted half data."""
        q = np.ascontiguousarray(q, np.float32)
        cells = np.zeros(self.K, np.int32)
        nc = np.zeros(1, np.int64)
        d1 = np.zeros(self.sk); d2 = np.zeros(self.sk)
        i1 = np.zeros(self.sk, np.int32); i2 = np.zeros(self.sk, np.int32)
        ap = lib().so_query_cells(self.h, _p(q), i, float(alpha), form, _p(cells), _p(nc),
                                  _p(d1), _p(d2), _p(i1), _p(i2))
        return cells[: nc[0]].copy(), int(ap), (d1, i1, d2, i2)

    def da(self, i, d1, i1, d2, i2, A, form=0):
        cells = np.zeros(self.K, np.int32)
        nc = np.zeros(1, np.int64)
        d1 = np.ascontiguousarray(d1, np.float64); d2 = np.ascontiguousarray(d2, np.float64)
        i1 = np.ascontiguousarray(i1, np.int32); i2 = np.ascontiguousarray(i2, np.int32)
        ap = lib().so_da(self.h, i, _p(d1), _p(i1), _p(d2), _p(i2), int(A), form, _p(cells), _p(nc))
        return cells[: nc[0]].copy(), int(ap)

    def da_trace(self, i, d1, i1, d2, i2, A):
        """Form 0 of Dynamic Activation (Alg. 3's retrieval order, walked row by row); also the
        number of first-half rows Alg. 3 has activated after each round."""
        cells = np.zeros(self.K, np.int32)
        trace = np.zeros(self.K, np.int32)
        nc = np.zeros(1, np.int64)
        d1 = np.ascontiguousarray(d1, np.float64); d2 = np.ascontiguousarray(d2, np.float64)
        i1 = np.ascontiguousarray(i1, np.int32); i2 = np.ascontiguousarray(i2, np.int32)
        ap = lib().so_da_trace(self.h, i, _p(d1), _p(i1), _p(d2), _p(i2), int(A), _p(cells),
                               _p(nc), _p(trace))
        return cells[: nc[0]].copy(), int(ap), trace[: nc[0]].copy()

    def query(self, Q, k, alpha, beta, form=0, want_scores=False, want_cand=False, nthreads=None):
        """Alg. 4 for every row of Q.  alpha: scalar or per-query array."""
        Q = np.ascontiguousarray(Q, np.float32).reshape(-1, self.d)
        nq = Q.shape[0]
        al = np.ascontiguousarray(np.broadcast_to(np.asarray(alpha, np.float64), (nq,)), np.float64)
        B = count_B(beta, self.n, k)
        ids = np.zeros((nq, k), np.int32)
        dists = np.zeros((nq, k), np.float64)
        sc = np.zeros((nq, self.n), np.uint8) if want_scores else None
        cand = np.zeros((nq, B), np.int32) if want_cand else None
        ncell = np.zeros((nq, self.ns), np.int64)
        ap = np.zeros((nq, self.ns), np.int64)
        rc = lib().so_query(self.h, _p(Q), nq, k, _p(al), float(beta), form, _p(ids), _p(dists),
                            _p(sc) if sc is not None else None, _p(cand) if cand is not None else None,
                            _p(ncell), _p(ap), nthreads or default_threads())
        assert rc == 0
        out = dict(ids=ids, dists=dists, ncells=ncell, aprime=ap)
        if sc is not None:
            out["scores"] = sc
        if cand is not None:
            out["cand"] = cand
        return out


def select(scores: np.ndarray, B: int) -> np.ndarray:
    s = np.ascontiguousarray(scores, np.uint8)
    out = np.zeros(B, np.int32)
    lib().so_select(_p(s), s.shape[0], B, _p(out))
    return out


def rerank(X, q, cand, k, metric=0):
    X = np.ascontiguousarray(X, np.float32)
    q = np.ascontiguousarray(q, np.float32)
    cand = np.ascontiguousarray(cand, np.int32)
    ids = np.zeros(k, np.int32)
    dist = np.zeros(k, np.float64)
    lib().so_rerank_metric(_p(X), X.shape[1], _p(q), _p(cand), cand.shape[0], k, int(metric), _p(ids), _p(dist))
    return ids, dist


def sclinear(X, ns, Q, k, alpha, beta, want_scores=False, nthreads=None, metric=0):
    X = np.ascontiguousarray(X, np.float32)
    Q = np.ascontiguousarray(Q, np.float32).reshape(-1, X.shape[1])
    n, d = X.shape
    nq = Q.shape[0]
    ids = np.zeros((nq, k), np.int32)
    dist = np.zeros((nq, k), np.float64)
    sc = np.zeros((nq, n), np.uint8) if want_scores else None
    lib().so_sclinear_metric(_p(X), n, d, ns, _p(Q), nq, k, float(alpha), float(beta), int(metric), _p(ids),
                             _p(dist), _p(sc) if sc is not None else None, nthreads or default_threads())
    return (ids, dist, sc) if want_scores else (ids, dist)


def bruteforce(X, Q, k, nthreads=None, metric=0):
    """Exact k-NN by (distance, id): Euclidean (metric 0) or Manhattan (metric 1)."""
    X = np.ascontiguousarray(X, np.float32)
    Q = np.ascontiguousarray(Q, np.float32).reshape(-1, X.shape[1])
    ids = np.zeros((Q.shape[0], k), np.int32)
    dist = np.zeros((Q.shape[0], k), np.float64)
    lib().so_bruteforce_metric(_p(X), X.shape[0], X.shape[1], _p(Q), Q.shape[0], k, int(metric), _p(ids),
                               _p(dist), nthreads or default_threads())
    return ids, dist


def bf16_round_arith(x) -> np.ndarray:
    """Round FP32 values to BF16 (nearest, ties to even), returned as FP32: the C
    oracle's arithmetic form (scale, nearbyint, scale back), used by its step-1 model."""
    x = np.ascontiguousarray(x, np.float32)
    out = np.empty_like(x)
    lib().so_bf16_round(_p(x), x.size, _p(out))
    return out


def recall(ids: np.ndarray, gt: np.ndarray) -> float:
    """Sec. 5.1: |R intersect R*| / k, averaged over queries."""
    k = gt.shape[1]
    return float(np.mean([len(set(a[:k].tolist()) & set(b.tolist())) / k for a, b in zip(ids, gt)]))


def mre(dists: np.ndarray, gt_dists: np.ndarray) -> float:
    """Sec. 5.1: mean over i of (|q,o_i| - |q,o_i*|) / |q,o_i*| (zero-distance terms skipped)."""
    g = np.asarray(gt_dists, np.float64)
    r = np.asarray(dists, np.float64)
    m = g > 0
    return float(np.mean(np.where(m, (r - g) / np.where(m, g, 1.0), 0.0)))


from .mlp import MLP64, gelu, bf16_round  # noqa: E402,F401
