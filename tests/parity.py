"""Comparison rules between the GPU path and the FP64 oracle.

Integer stages (SC-scores, candidate sets, activated cells) must match
exactly.  The only tolerated difference is at a floating-point tie: the GPU
ranks cells by FP32 keys and candidates by FP32 distances, the oracle by FP64.

 * Cells: for a (query, subspace) the two activated sets may differ only in
   "band" cells, whose FP64 key is within 1e-5 (relative) of the oracle's
   cutoff key.  Where that happens the scores of the affected points may
   differ; the GPU's scores must then equal the counts over its own activated
   cells in the oracle's inverted multi-index (Def. 4 on those cells), its A'
   their summed sizes, and the oracle's selection and re-rank, re-run on those
   scores, must give the GPU's candidates and top-k.
 * Top-k: ids must be identical unless distances tie within 1e-5 relative;
   in that case the GPU's list must be a valid top-k: its FP64 distances must
   equal the oracle's sorted top-k distances within 1e-5 relative.
"""
from __future__ import annotations

import numpy as np

import oracle

REL = 1e-5


def cells_to_gpu_layout(ref_cells, nq, ns, K):
    """Oracle activated cells [q][i] -> (uint16 [nq][ns][K], int32 [nq][ns])."""
    cells = np.zeros((nq, ns, K), np.uint16)
    ncell = np.zeros((nq, ns), np.int32)
    for q in range(nq):
        for i in range(ns):
            c = ref_cells[q][i]
            cells[q, i, :len(c)] = c
            ncell[q, i] = len(c)
    return cells, ncell


def oracle_cells(oix, Q, alpha, form=0):
    """Per (query, subspace): (cells, A', keys of every cell by id, cutoff key)."""
    out = []
    sk = oix.sk
    al = np.broadcast_to(np.asarray(alpha, np.float64), (Q.shape[0],))
    for q in range(Q.shape[0]):
        row = []
        for i in range(oix.ns):
            cells, ap, (d1, i1, d2, i2) = oix.cells(Q[q], i, float(al[q]), form)
            key = (d1[:, None] + d2[None, :]).reshape(-1)     # key of cell c1*sk + c2
            row.append((cells, ap, key, key[cells[-1]]))
        out.append(row)
    return out


def check_cells(ref, gpu_cells, gpu_ncells, q, i, extra=0.0):
    """Returns True if identical, False if they differ only in band cells; raises otherwise.
    `extra` widens the band by an absolute key tolerance (keys computed in lower precision)."""
    cells, ap, key, kstar = ref[q][i]
    g = set(gpu_cells[q, i, :gpu_ncells[q, i]].tolist())
    o = set(cells.tolist())
    if g == o:
        return True
    diff = g ^ o
    band = np.abs(key[list(diff)] - kstar) <= REL * max(kstar, 1e-30) + extra
    assert band.all(), f"query {q} subspace {i}: cells differ outside the tie band: {sorted(diff)[:10]}"
    return False


def true_dists(X64, ids, q, metric=0):
    """FP64 distances of rows `ids` to q: Euclidean, or Manhattan (metric 1)."""
    diff = X64[ids] - q.astype(np.float64)
    return np.abs(diff).sum(axis=1) if metric else np.sqrt((diff ** 2).sum(axis=1))


def check_topk(X, Q, ids, dists, ref_ids, ref_dists, k, metric=0):
    """Top-k identical, or a valid top-k under distance ties within REL."""
    X64 = X.astype(np.float64)
    for q in range(Q.shape[0]):
        if np.array_equal(ids[q], ref_ids[q]):
            assert np.allclose(dists[q], ref_dists[q], rtol=REL, atol=1e-6), f"query {q}: distances"
            continue
        true = true_dists(X64, ids[q], Q[q], metric)
        assert len(set(ids[q].tolist())) == k, f"query {q}: repeated ids"
        assert np.allclose(np.sort(true), np.sort(ref_dists[q]), rtol=REL, atol=1e-6), \
            f"query {q}: ids {ids[q]} vs {ref_ids[q]} not a tie"
        assert np.allclose(dists[q], true, rtol=REL, atol=1e-6)


def scores_from_cells(oix, gpu_cells, gpu_ncells, q):
    """SC-scores of query q counted over the given activated cells in the
    oracle's IMI (a point scores once per subspace whose activated cells hold
    it), and the points in those cells per subspace."""
    if not hasattr(oix, "_imi"):
        oix._imi = (oix.offs(), oix.ids())
    offs, ids = oix._imi
    sc = np.zeros(oix.n, np.int64)
    sizes = np.zeros(oix.ns, np.int64)
    for i in range(oix.ns):
        for c in gpu_cells[q, i, :gpu_ncells[q, i]].tolist():
            a, b = int(offs[i, c]), int(offs[i, c + 1])
            sc[ids[i, a:b]] += 1
            sizes[i] += b - a
    return sc, sizes


def check_query(oix, X, Q, k, alpha, beta, gpu, key_tol=None):
    """Full comparison of a GPU query_debug result with the oracle.  Returns stats.
    key_tol [nq][ns], if given, widens each (query, subspace) band by that absolute amount."""
    nq = Q.shape[0]
    ref = oix.query(Q, k, alpha, beta, want_scores=True, want_cand=True)
    rc = oracle_cells(oix, Q, alpha)
    B = oracle.count_B(beta, oix.n, k)
    g_sc = gpu["scores"]
    n_band = 0
    for q in range(nq):
        exact = all(check_cells(rc, gpu["cells"], gpu["ncells"], q, i,
                                0.0 if key_tol is None else float(key_tol[q, i])) for i in range(oix.ns))
        assert np.array_equal(gpu["aprime"][q], ref["aprime"][q]) or not exact
        if exact:
            assert np.array_equal(g_sc[q], ref["scores"][q]), f"query {q}: SC-scores differ"
            assert np.array_equal(np.sort(gpu["cand"][q]), np.sort(ref["cand"][q])), f"query {q}: candidates"
            check_topk(X, Q[q:q + 1], gpu["ids"][q:q + 1], gpu["dists"][q:q + 1], ref["ids"][q:q + 1],
                       ref["dists"][q:q + 1], k, oix.metric)
        else:
            n_band += 1
            # the GPU's scores are the counts over its own cells, A' their sizes
            sc, sizes = scores_from_cells(oix, gpu["cells"], gpu["ncells"], q)
            assert np.array_equal(g_sc[q].astype(np.int64), sc), f"query {q}: SC-scores of its own cells"
            assert np.array_equal(np.asarray(gpu["aprime"][q], np.int64), sizes), f"query {q}: A'"
            # conditional parity: the oracle's selection and re-rank on the GPU's scores
            c = oracle.select(g_sc[q], B)
            assert np.array_equal(np.sort(gpu["cand"][q]), np.sort(c)), f"query {q}: conditional candidates"
            r_ids, r_d = oracle.rerank(X, Q[q], c, k, oix.metric)
            check_topk(X, Q[q:q + 1], gpu["ids"][q:q + 1], gpu["dists"][q:q + 1], r_ids[None], r_d[None], k,
                       oix.metric)
    rec_gpu = oracle.recall(gpu["ids"], ref["ids"])
    return dict(band_queries=n_band, ref=ref, agree=rec_gpu)
