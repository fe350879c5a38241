"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each check below is computed independently of the oracle's own code (NumPy
brute force, closed forms, the paper's worked example, invariants), so that a
dropped term, a wrong index or a transposed operand in the oracle fails one.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- helpers --
def np_knn(X, q, k, ids=None):
    """Exact k-NN by (squared distance, id), NumPy FP64."""
    X64 = X.astype(np.float64)
    d2 = ((X64 - q.astype(np.float64)) ** 2).sum(axis=1)
    if ids is None:
        ids = np.arange(X.shape[0])
    else:
        d2 = d2[ids]
    order = np.lexsort((ids, d2))[:k]
    return np.asarray(ids)[order], np.sqrt(d2[order])


def small_index(n=600, d=16, ns=4, sk=4, seed=3, kind="clustered", iters=10):
    X = synth.tiny(n, d, seed, kind, levels=4)
    c64, c32, asg, obj = oracle.build_index(X, ns, sk, iters=iters, seed=seed)
    return X, oracle.Index(X, ns, sk, c32, asg), (c64, c32, asg, obj)


def grid_index(sk, sizes):
    """An oracle index whose IMI cell c = a1*sk + a2 holds sizes[c] points."""
    a1, a2 = [], []
    for c, m in enumerate(sizes):
        a1 += [c // sk] * m
        a2 += [c % sk] * m
    n = len(a1)
    X = np.zeros((n, 2), np.float32)
    asg = np.stack([np.array(a1, np.int32), np.array(a2, np.int32)])
    cent = np.zeros(sk * 2, np.float32)
    return oracle.Index(X, 1, sk, cent, asg)


# ------------------------------------------------------------- counts/layout
def test_counts_A_B():
    # Alg. 3 stop rule and Alg. 1/4 candidate loop at the workloads' settings
    assert oracle.count_A(0.03, 1_000_000) == 30_000        # 0.03*1e6 is 30000.000000000004 in FP64
    assert oracle.count_A(0.05, 10_000) == 500
    assert oracle.count_A(0.01, 1_000_000) == 10_000
    assert oracle.count_A(0.02, 10_000_000) == 200_000
    assert oracle.count_A(1e-9, 100) == 1                  # at least one point
    assert oracle.count_A(1.0, 77) == 77
    assert oracle.count_A(0.0301, 1000) == 31              # ceiling
    assert oracle.count_B(0.005, 1_000_000, 10) == 5_000
    assert oracle.count_B(0.005, 10_000, 10) == 50
    assert oracle.count_B(0.001, 10_000, 50) == 50         # raised to k
    assert oracle.count_B(0.0059, 1000, 1) == 5            # floor
    assert oracle.count_B(1.0, 123, 5) == 123


def test_layout_contiguous_division():
    # Sec. 3.2 contiguous division; Def. 3: the last subspace takes the remainder
    d0, w = oracle.layout(128, 8)
    assert list(d0) == [8 * g for g in range(16)] and set(w) == {8}
    d0, w = oracle.layout(10, 3)
    assert list(d0) == [0, 1, 3, 4, 6, 8] and list(w) == [1, 2, 1, 2, 2, 2]
    d0, w = oracle.layout(960, 20)
    assert set(w) == {24} and d0[-1] == 960 - 24
    d0, w = oracle.layout(96, 8)
    assert set(w) == {6}


# ------------------------------------------------------- Dynamic Activation --
def test_da_worked_example_fig5():
    g = json.load(open(os.path.join(GOLDEN, "da_fig5.json")))
    ix = grid_index(3, [1] * 9)
    d1, d2 = np.array(g["dists1"]), np.array(g["dists2"])
    ident = np.arange(3, dtype=np.int32)
    cells, ap, trace = ix.da_trace(0, d1, ident, d2, ident, A=9)
    for r, (a, b, key) in enumerate(g["first_rounds"]):
        assert divmod(int(cells[r]), 3) == (a, b)
        assert abs(d1[a] + d2[b] - key) < 1e-12
    assert list(trace[:3]) == g["active_rows_after_round"]
    assert ap == 9 and len(cells) == 9 and sorted(cells) == list(range(9))
    # stop rule: A=2 stops after round 2 (two unit cells)
    cells2, ap2, _ = ix.da_trace(0, d1, ident, d2, ident, A=2)
    assert list(cells2) == [0, 3] and ap2 == 2


@pytest.mark.parametrize("seed", range(12))
def test_da_three_forms_agree_with_numpy_prefix(seed):
    rng = np.random.default_rng(seed)
    sk = int(rng.integers(1, 9))
    sizes = rng.integers(0, 5, size=sk * sk)
    sizes[rng.integers(0, sk * sk)] += 1                  # n >= 1
    ix = grid_index(sk, sizes.tolist())
    n = int(sizes.sum())
    if seed % 2:
        d1 = rng.integers(0, 4, size=sk).astype(np.float64)   # forces key ties
        d2 = rng.integers(0, 4, size=sk).astype(np.float64)
    else:
        d1, d2 = rng.random(sk), rng.random(sk)
    i1 = np.lexsort((np.arange(sk), d1)).astype(np.int32)
    i2 = np.lexsort((np.arange(sk), d2)).astype(np.int32)
    for A in sorted({1, max(1, n // 3), max(1, n // 2), n}):
        res = [ix.da(0, d1, i1, d2, i2, A, form=f) for f in (0, 1, 2)]
        for cells, ap in res[1:]:
            assert np.array_equal(cells, res[0][0]) and ap == res[0][1]
        # independent: lexicographic (key, r1, r2) order, shortest prefix reaching A
        r1, r2 = np.meshgrid(np.arange(sk), np.arange(sk), indexing="ij")
        key = d1[i1][r1] + d2[i2][r2]
        order = np.lexsort((r2.ravel(), r1.ravel(), key.ravel()))
        cellid = (i1[r1] * sk + i2[r2]).ravel()[order]
        cum = np.cumsum(sizes[cellid])
        m = int(np.searchsorted(cum, A) + 1)
        assert np.array_equal(res[0][0], cellid[:m])
        assert res[0][1] == cum[m - 1] >= A
        assert m == 1 or cum[m - 2] < A


# ------------------------------------------------------ SC-Linear (Alg. 1) --
@pytest.mark.parametrize("seed,kind", [(1, "gauss"), (2, "int"), (3, "clustered")])
def test_sclinear_scores_equal_def4_rank_count(seed, kind):
    X = synth.tiny(300, 12, seed, kind, levels=3)
    Q = synth.tiny(4, 12, seed + 100, kind, levels=3)
    ns, alpha = 3, 0.1
    A = oracle.count_A(alpha, 300)
    _, _, sc = oracle.sclinear(X, ns, Q, 5, alpha, 0.05, want_scores=True)
    d0, w = oracle.layout(12, ns)
    for qi, q in enumerate(Q):
        expect = np.zeros(300, np.int64)
        for i in range(ns):
            lo, hi = d0[2 * i], d0[2 * i] + w[2 * i] + w[2 * i + 1]
            dsub = ((X[:, lo:hi].astype(np.float64) - q[lo:hi]) ** 2).sum(axis=1)
            # rank_i(o) = #{o' : (d(o'), id') < (d(o), id)}, by pairwise comparison
            less = (dsub[None, :] < dsub[:, None]) | ((dsub[None, :] == dsub[:, None]) &
                                                      (np.arange(300)[None, :] < np.arange(300)[:, None]))
            rank = less.sum(axis=1)
            expect += rank < A
        assert np.array_equal(sc[qi].astype(np.int64), expect)


def test_sclinear_single_subspace_is_exact_knn():
    # Def. 1: with one subspace covering all d dims and A = B = k, the k colliding
    # points are exactly the k nearest
    X = synth.tiny(500, 10, 7, "gauss")
    Q = synth.tiny(5, 10, 8, "gauss")
    k = 7
    ids, dist = oracle.sclinear(X, 1, Q, k, k / 500, k / 500)
    for qi, q in enumerate(Q):
        e_ids, e_d = np_knn(X, q, k)
        assert np.array_equal(ids[qi], e_ids)
        assert np.allclose(dist[qi], e_d, rtol=1e-12)


# ----------------------------------------------------- SuCo (Alg. 2, 3, 4) --
@pytest.mark.parametrize("kind", ["gauss", "int", "clustered"])
def test_alpha_beta_one_reduces_to_exact_search(kind):
    X, ix, _ = small_index(kind=kind)
    Q = synth.tiny(6, 16, 99, kind, levels=4)
    k = 8
    out = ix.query(Q, k, 1.0, 1.0)
    ids_l, d_l = oracle.sclinear(X, 4, Q, k, 1.0, 1.0)
    for qi, q in enumerate(Q):
        e_ids, e_d = np_knn(X, q, k)
        assert np.array_equal(out["ids"][qi], e_ids)
        assert np.array_equal(ids_l[qi], e_ids)
        assert np.allclose(out["dists"][qi], e_d, rtol=1e-12)


@pytest.mark.parametrize("alpha", [0.01, 0.1, 0.4])
def test_beta_one_exact_for_any_alpha(alpha):
    X, ix, _ = small_index(kind="gauss", seed=5)
    Q = synth.tiny(4, 16, 55, "gauss")
    out = ix.query(Q, 5, alpha, 1.0)
    for qi, q in enumerate(Q):
        assert np.array_equal(out["ids"][qi], np_knn(X, q, 5)[0])


def test_alpha_one_all_scores_ns_and_lowest_ids_selected():
    X, ix, _ = small_index(kind="clustered", seed=9)
    Q = synth.tiny(3, 16, 77, "clustered")
    beta, k = 0.05, 4
    B = oracle.count_B(beta, 600, k)
    out = ix.query(Q, k, 1.0, beta, want_scores=True, want_cand=True)
    assert (out["scores"] == 4).all()
    for qi, q in enumerate(Q):
        assert list(out["cand"][qi]) == list(range(B))
        assert np.array_equal(out["ids"][qi], np_knn(X, q, k, ids=np.arange(B))[0])


def test_single_cell_index_degenerates_like_alpha_one():
    X = synth.tiny(200, 8, 4, "gauss")
    c64, c32, asg, _ = oracle.build_index(X, 2, 1, iters=3)
    assert (asg == 0).all()
    ix = oracle.Index(X, 2, 1, c32, asg)
    out = ix.query(synth.tiny(2, 8, 5, "gauss"), 3, 0.05, 0.1, want_scores=True, want_cand=True)
    assert (out["scores"] == 2).all()
    assert list(out["cand"][0]) == list(range(20))


@pytest.mark.parametrize("kind", ["gauss", "int"])
def test_suco_scores_count_activated_cells(kind):
    X, ix, (c64, c32, asg, _) = small_index(kind=kind, seed=11)
    Q = synth.tiny(5, 16, 12, kind, levels=4)
    ns, sk, n = 4, 4, 600
    d0, w = oracle.layout(16, ns)
    cent = c32.astype(np.float64)
    prev = None
    for alpha in (0.02, 0.1, 0.3):
        A = oracle.count_A(alpha, n)
        out = ix.query(Q, 5, alpha, 0.05, want_scores=True)
        assert (out["scores"].sum(axis=1) == out["aprime"].sum(axis=1)).all()
        for qi, q in enumerate(Q):
            expect = np.zeros(n, np.int64)
            for i in range(ns):
                # independent DA: centre distances, rank, lexicographic prefix
                dh = []
                for h in range(2):
                    g = 2 * i + h
                    C = cent[sk * d0[g]: sk * (d0[g] + w[g])].reshape(sk, w[g])
                    dh.append(((C - q[d0[g]:d0[g] + w[g]].astype(np.float64)) ** 2).sum(axis=1))
                cell = asg[2 * i] * sk + asg[2 * i + 1]
                size = np.bincount(cell, minlength=sk * sk)
                o1 = np.lexsort((np.arange(sk), dh[0]))
                o2 = np.lexsort((np.arange(sk), dh[1]))
                r1, r2 = np.meshgrid(np.arange(sk), np.arange(sk), indexing="ij")
                key = dh[0][o1][r1] + dh[1][o2][r2]
                order = np.lexsort((r2.ravel(), r1.ravel(), key.ravel()))
                cid = (o1[r1] * sk + o2[r2]).ravel()[order]
                cum = np.cumsum(size[cid])
                m = int(np.searchsorted(cum, A) + 1)
                act = np.zeros(sk * sk, bool)
                act[cid[:m]] = True
                expect += act[cell]
                assert out["aprime"][qi, i] == cum[m - 1] >= A
                assert cum[m - 1] - size[cid[m - 1]] < A
            assert np.array_equal(out["scores"][qi].astype(np.int64), expect)
        if prev is not None:
            assert (out["scores"] >= prev).all()          # non-decreasing in alpha
        prev = out["scores"]


def test_da_forms_give_identical_queries():
    X, ix, _ = small_index(kind="int", seed=21)
    Q = synth.tiny(6, 16, 22, "int", levels=4)
    outs = [ix.query(Q, 5, 0.07, 0.05, form=f, want_scores=True) for f in (0, 1, 2)]
    for o in outs[1:]:
        assert np.array_equal(o["scores"], outs[0]["scores"])
        assert np.array_equal(o["ids"], outs[0]["ids"])


# ------------------------------------------------------- select / re-rank --
@pytest.mark.parametrize("seed", range(5))
def test_select_properties(seed):
    rng = np.random.default_rng(seed)
    n, ns = 997, 6
    s = rng.integers(0, ns + 1, size=n).astype(np.uint8)
    for B in (1, 10, 100, 500, n):
        c = oracle.select(s, B)
        assert len(c) == B == len(set(c.tolist()))
        inside = np.zeros(n, bool)
        inside[c] = True
        if B < n:
            T = s[inside].min()
            assert T >= s[~inside].max()
            # among points scoring exactly T, the lowest ids are taken
            eq = np.flatnonzero(s == T)
            take = inside[eq]
            assert take[: take.sum()].all() and not take[take.sum():].any()


def test_rerank_is_bruteforce_over_candidates():
    X = synth.tiny(400, 9, 31, "int", levels=3)          # many exact distance ties
    q = synth.tiny(1, 9, 32, "int", levels=3)[0]
    cand = np.random.default_rng(0).choice(400, 120, replace=False).astype(np.int32)
    ids, dist = oracle.rerank(X, q, cand, 15)
    e_ids, e_d = np_knn(X, q, 15, ids=cand)
    assert np.array_equal(ids, e_ids)
    assert np.array_equal(dist, e_d)


def test_bruteforce_matches_numpy():
    X = synth.tiny(300, 7, 41, "gauss")
    Q = synth.tiny(4, 7, 42, "gauss")
    ids, dist = oracle.bruteforce(X, Q, 6)
    for qi, q in enumerate(Q):
        e_ids, e_d = np_knn(X, q, 6)
        assert np.array_equal(ids[qi], e_ids)
        assert np.allclose(dist[qi], e_d, rtol=1e-13)


# --------------------------------------------------------- index (Alg. 2) --
def test_kmeans_invariants():
    X = synth.tiny(800, 6, 51, "clustered")
    d0, w = oracle.layout(6, 1)
    init = oracle.init_ids(X, 1, 5, 1, 0)
    assert len(set(init.tolist())) == 5
    cent, asg, obj = oracle.kmeans(X, int(d0[0]), int(w[0]), 5, 30, init)
    # Lloyd never increases the objective
    assert (np.diff(obj) <= 1e-9 * obj[0]).all()
    # final assignment is the argmin with lowest-id ties
    H = X[:, d0[0]:d0[0] + w[0]].astype(np.float64)
    D = ((H[:, None, :] - cent[None, :, :]) ** 2).sum(axis=2)
    assert np.array_equal(asg, np.argmin(D, axis=1))
    assert np.bincount(asg, minlength=5).sum() == 800
    assert abs(obj[-1] - D.min(axis=1).sum()) <= 1e-9 * obj[-1]
    # at a fixed point every centre is the mean of its members
    if obj[-1] == obj[-2]:
        for c in range(5):
            m = asg == c
            if m.any():
                assert np.allclose(cent[c], H[m].mean(axis=0), rtol=1e-12, atol=1e-12)


def test_kmeans_update_exact_means_across_sum_groups():
    """Integer data, clusters of several hundred members (more than one
    summation group, a ragged last group): every FP64 partial sum is an exact
    integer, so after one update each centre is exactly the exact mean rounded
    once (sum / m), whatever the grouping; a dropped or doubled group fails."""
    rng = np.random.default_rng(12)
    lab = rng.integers(0, 3, 2000)
    X = (np.array([[0, 0], [100, 0], [0, 100]])[lab] + rng.integers(-20, 21, (2000, 2))).astype(np.float32)
    init = np.array([np.flatnonzero(lab == c)[0] for c in range(3)], np.int64)
    cent, asg, _ = oracle.kmeans(X, 0, 2, 3, 1, init)
    H = X.astype(np.float64)
    a0 = np.argmin(((H[:, None, :] - H[init][None, :, :]) ** 2).sum(axis=2), axis=1)
    for c in range(3):
        m = int((a0 == c).sum())
        assert m > 256 and m % 256
        tot = [sum(int(v) for v in X[a0 == c, j]) for j in range(2)]
        assert np.array_equal(cent[c], np.array(tot, np.float64) / m)


def test_kmeans_separates_obvious_clusters():
    rng = np.random.default_rng(0)
    centres = np.array([[-10.0, 0.0], [0.0, 10.0], [10.0, 0.0]])
    lab = rng.integers(0, 3, 600)
    X = (centres[lab] + 0.1 * rng.normal(size=(600, 2))).astype(np.float32)
    # one initial centre inside each cluster: Lloyd must then recover the labels
    init = np.array([np.flatnonzero(lab == c)[0] for c in (2, 0, 1)], np.int64)
    cent, a, obj = oracle.kmeans(X, 0, 2, 3, 20, init)
    assert np.array_equal(a, np.array([1, 2, 0])[lab])
    assert np.allclose(cent, centres[[2, 0, 1]], atol=0.05)


def test_imi_invariants():
    X, ix, (c64, c32, asg, obj) = small_index(kind="gauss", seed=61)
    offs, ids = ix.offs(), ix.ids()
    sk, ns, n = 4, 4, 600
    assert np.array_equal(c32, c64.astype(np.float32))
    for i in range(ns):
        assert offs[i, 0] == 0 and offs[i, -1] == n and (np.diff(offs[i]) >= 0).all()
        assert np.array_equal(np.sort(ids[i]), np.arange(n))
        cell = asg[2 * i] * sk + asg[2 * i + 1]
        for c in range(sk * sk):
            mem = ids[i, offs[i, c]:offs[i, c + 1]]
            assert (np.diff(mem) > 0).all()
            assert (cell[mem] == c).all()
            assert len(mem) == (cell == c).sum()


def test_centroid_dists_closed_form():
    X, ix, (c64, c32, asg, _) = small_index(kind="gauss", seed=71)
    q = synth.tiny(1, 16, 72, "gauss")[0]
    d0, w = oracle.layout(16, 4)
    for g in range(8):
        C = c32[4 * d0[g]: 4 * (d0[g] + w[g])].reshape(4, w[g]).astype(np.float64)
        e = ((C - q[d0[g]:d0[g] + w[g]]) ** 2).sum(axis=1)
        assert np.allclose(ix.centroid_dists(q, g), e, rtol=1e-14)


# ------------------------------------------------- paper's qualitative claim
def test_scores_favour_true_neighbours():
    # Sec. 3.3: points closer to the query tend to have larger SC-scores
    W = synth.Workload(1)
    X = W.data(3000)
    Q = W.queries(8)
    _, c32, asg, _ = oracle.build_index(X, 8, 8, iters=8)
    ix = oracle.Index(X, 8, 8, c32, asg)
    out = ix.query(Q, 10, 0.1, 0.02, want_scores=True)
    for qi, q in enumerate(Q):
        nn, _ = np_knn(X, q, 10)
        assert out["scores"][qi][nn].mean() > out["scores"][qi].mean() + 2.0


# ------------------------------------------------------------- MLP / BF16 --
def test_gelu_values():
    assert oracle.gelu(np.array([0.0]))[0] == 0.0
    assert abs(oracle.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15     # Phi(1)
    assert abs(oracle.gelu(np.array([-1.0]))[0] + 0.15865525393145707) < 1e-15   # -Phi(-1)


def test_mlp_gradient_matches_central_differences():
    from oracle.mlp import MLP64, init_params, PARAM_NAMES
    rng = np.random.default_rng(0)
    p = init_params(5, 7, seed=3)
    for k in p:
        p[k] = p[k] + 0.1 * rng.normal(size=p[k].shape)   # non-zero biases too
    net = MLP64(p, mu=rng.normal(size=5), sigma=1.0 + rng.random(5))
    F = rng.normal(size=(9, 5))
    t = rng.normal(size=9)
    _, g = net.loss_and_grad(F, t)
    h = 1e-6
    for name in PARAM_NAMES:
        flat = net.p[name].reshape(-1)
        for j in range(flat.size):
            old = flat[j]
            flat[j] = old + h
            lp, _ = net.loss_and_grad(F, t)
            flat[j] = old - h
            lm, _ = net.loss_and_grad(F, t)
            flat[j] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name].reshape(-1)[j]) <= 1e-6 * max(1.0, abs(fd))


def test_adam_first_step_moves_by_lr():
    # Kingma & Ba: with bias correction the first step is lr * sign(g) (up to eps)
    from oracle.mlp import MLP64, init_params
    net = MLP64(init_params(3, 4, seed=1))
    before = {k: v.copy() for k, v in net.p.items()}
    g = {k: np.full_like(v, 0.5) for k, v in net.p.items()}
    net.adam_step(g, {}, lr=1e-3)
    for k in net.p:
        assert np.allclose(before[k] - net.p[k], 1e-3, rtol=1e-6)


def test_bf16_round_to_nearest_even():
    import torch
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.5, 3.14159, 1e-30, 65504.0, 0.0], np.float32)
    r = oracle.bf16_round(vals)
    assert r[1] == 1.0 and r[2] == np.float32(1.015625)
    t = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(r, t)
    x = np.random.default_rng(0).normal(size=10000).astype(np.float32) * 100
    assert np.array_equal(oracle.bf16_round(x),
                          torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy())


def test_bf16_arith_form_matches_bit_form_and_torch():
    # the C oracle rounds arithmetically, oracle.mlp by bit arithmetic, torch by its own conversion
    import torch
    rng = np.random.default_rng(7)
    x = (rng.standard_normal(200000) * 10.0 ** rng.integers(-44, 38, 200000)).astype(np.float32)
    ties = (np.float32(1.0) + np.arange(1, 512, 2, dtype=np.float32) * np.float32(2 ** -8)).astype(np.float32)
    sub = (np.arange(-300, 300, dtype=np.float32) * np.float32(2 ** -140)).astype(np.float32)
    big = np.array([3.3895314e38, 3.3961775e38, 3.40282e38, -3.40282e38, np.inf, -np.inf, 0.0, -0.0], np.float32)
    allv = np.concatenate([x, ties, sub, big]).astype(np.float32)
    a = oracle.bf16_round_arith(allv)
    b = oracle.bf16_round(allv)
    t = torch.from_numpy(allv).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(a.view(np.uint32), t.view(np.uint32))
    assert np.array_equal(b.view(np.uint32), t.view(np.uint32))
    # relative rounding error at most 2^-8 for normal values
    nz = (np.abs(allv) > 2.0 ** -126) & np.isfinite(allv) & np.isfinite(a)
    assert (np.abs(a[nz].astype(np.float64) - allv[nz]) <= 2.0 ** -8 * np.abs(allv[nz].astype(np.float64))).all()


def test_s1_bf16_model_equals_fp32_on_bf16_exact_values():
    # values with at most 8 significant bits are unchanged by BF16 rounding, so the
    # split-precision step-1 model must reproduce the plain step-1 distances exactly
    X = (np.random.default_rng(3).integers(0, 64, size=(400, 16)) / 4.0).astype(np.float32)
    c64, c32, asg, _ = oracle.build_index(X, 4, 4, iters=5, seed=2)
    c32 = oracle.bf16_round(c32)            # make the centres BF16-exact too
    ix = oracle.Index(X, 4, 4, c32, asg)
    q = X[17] + np.float32(0.25)
    plain = [ix.centroid_dists(q, g) for g in range(8)]
    ix.set_s1_bf16(True)
    model = [ix.centroid_dists(q, g) for g in range(8)]
    for a, b in zip(plain, model):
        assert np.array_equal(a, b)


def test_s1_bf16_model_is_distance_of_rounded_values():
    import torch
    X, ix, (c64, c32, asg, _) = small_index(n=500, d=24, ns=3, sk=5, seed=11, kind="gauss")
    q = (X[3] * np.float32(1.37) + np.float32(0.011)).astype(np.float32)
    ix.set_s1_bf16(True)
    lay = oracle.layout(24, 3)
    for g in range(6):
        d0, w = int(lay[0][g]), int(lay[1][g])
        cen = c32.reshape(-1)[5 * d0:5 * d0 + 5 * w].reshape(5, w)
        qb = torch.from_numpy(q[d0:d0 + w].copy()).to(torch.bfloat16).double().numpy()
        cb = torch.from_numpy(cen.copy()).to(torch.bfloat16).double().numpy()
        ref = ((cb - qb[None, :]) ** 2).sum(axis=1)
        assert np.allclose(ix.centroid_dists(q, g), ref, rtol=1e-15, atol=0)
        # and differs from the FP32 distances by at most the rounding's effect
        ix.set_s1_bf16(False)
        plain = ix.centroid_dists(q, g)
        ix.set_s1_bf16(True)
        bound = 2 * np.sqrt(plain) * (2.0 ** -8) * (np.linalg.norm(q[d0:d0 + w]) + np.linalg.norm(cen, axis=1)) \
            + ((2.0 ** -8) * (np.linalg.norm(q[d0:d0 + w]) + np.linalg.norm(cen, axis=1))) ** 2
        assert (np.abs(ix.centroid_dists(q, g) - plain) <= bound * (1 + 1e-9)).all()


def test_theorem1_higher_score_means_closer_with_probability():
    # Thm. 1: for independent random points o1, o2 with SC-score(o1) > SC-score(o2),
    # ||o1 - q|| < ||o2 - q|| with probability at least 1/2 - 1/e^2 for suitable N_s and
    # alpha.  Checked on i.i.d. Gaussian data (independent subspace distances) with
    # SC-Linear's exact scores (Alg. 1), over all such pairs of points.
    rng = np.random.default_rng(12)
    X = rng.standard_normal((2000, 32)).astype(np.float32)
    Q = rng.standard_normal((4, 32)).astype(np.float32)
    _, _, sc = oracle.sclinear(X, 8, Q, 10, 0.1, 0.05, want_scores=True)
    bound = 0.5 - np.exp(-2.0)
    for qi, q in enumerate(Q):
        s = sc[qi].astype(np.int64)
        dist = np.sqrt(((X.astype(np.float64) - q) ** 2).sum(axis=1))
        higher = s[:, None] > s[None, :]
        closer = dist[:, None] < dist[None, :]
        frac = (higher & closer).sum() / higher.sum()
        assert frac >= bound, (qi, frac)
        assert frac > 0.5   # better than chance: inverted or shuffled scores fail here


def test_adam_steps_closed_form_over_three_steps():
    # Kingma & Ba, Algorithm 1, for a gradient sequence whose moments have closed
    # forms: g, then 0, then 0.  After step t the bias-corrected moments are
    #   t=1: m^ = g,                           v^ = g^2
    #   t=2: m^ = b1 (1-b1) g / (1-b1^2),      v^ = b2 (1-b2) g^2 / (1-b2^2)
    #   t=3: m^ = b1^2 (1-b1) g / (1-b1^3),    v^ = b2^2 (1-b2) g^2 / (1-b2^3)
    # A wrong decay, a missing or misplaced bias correction, or eps inside the
    # root changes the steps of t = 2 and 3 (t = 1 alone cannot tell them apart).
    from oracle.mlp import MLP64, init_params
    b1, b2, eps, lr = 0.9, 0.999, 1e-8, 1e-3
    net = MLP64(init_params(3, 4, seed=2))
    start = {k: v.copy() for k, v in net.p.items()}
    rng = np.random.default_rng(5)
    g = {k: rng.choice([-1.0, 1.0], size=v.shape) * (0.1 + rng.random(v.shape)) for k, v in net.p.items()}
    zero = {k: np.zeros_like(v) for k, v in net.p.items()}
    state = {}
    moved = {k: np.zeros_like(v) for k, v in net.p.items()}
    for t, gt in enumerate([g, zero, zero], start=1):
        before = {k: v.copy() for k, v in net.p.items()}
        net.adam_step(gt, state, lr=lr, b1=b1, b2=b2, eps=eps)
        for k in net.p:
            a = np.abs(g[k])
            mh = g[k] * b1 ** (t - 1) * (1 - b1) / (1 - b1 ** t)
            vh = a * a * b2 ** (t - 1) * (1 - b2) / (1 - b2 ** t)
            step = lr * mh / (np.sqrt(vh) + eps)
            assert np.allclose(before[k] - net.p[k], step, rtol=1e-9, atol=0), (t, k)
            moved[k] += step
    for k in net.p:
        assert np.allclose(start[k] - net.p[k], moved[k], rtol=1e-9, atol=0)
    # constant gradient: m^ = g and v^ = g^2 at every step, so t steps move lr*t*g/(|g|+eps)
    net2 = MLP64(init_params(3, 4, seed=2))
    st2 = {}
    for _ in range(4):
        net2.adam_step(g, st2, lr=lr)
    for k in net2.p:
        assert np.allclose(start[k] - net2.p[k], 4 * lr * g[k] / (np.abs(g[k]) + eps), rtol=1e-9, atol=0)


def _tiny_net_for_rounding_points():
    """A 1 -> 3 -> 3 -> 1 network whose BF16 inference value follows by hand.

    F = 1 + 2^-10 (an FP32 value; BF16 rounds it to 1).  Near 9 the BF16 spacing
    is 2^-4 and GELU(z) = z exactly in FP64 (1 - Phi(9) is far below 2^-53).
      unit 0: z1 = 2^-5 x + 9      -> 9 + 2^-5 at x = 1, the tie between 9 and
              9.0625, which rounds to the even 9; the unrounded x gives 9.0625
      unit 1: z1 = 2^-6 x + 9      -> 9.015625, rounded to 9
      unit 2: z1 = 0               -> 0
      layer 2 (h1 -> z2): z2 = [h1_0, h1_1 + 3*2^-7, h1_1 + 2^-7]
              with h1 = [9, 9, 0]: [9, 9.0234375, 9.0078125], all rounded to 9;
              an unrounded h1_1 = 9.015625 would give 9.0390625 -> 9.0625
      output: y = (1 + 2^-9) h2_0 + 2 h2_1 + 4 h2_2 + 0.5, where BF16 rounds
              1 + 2^-9 to 1, so y = 9 + 18 + 36 + 0.5 = 63.5.
    Each left-out rounding gives another value: the input (63.5625), h1
    (63.625), h2 (63.578125), the weights (63.517578125)."""
    from oracle.mlp import MLP64
    p = dict(W1=np.array([[2.0 ** -5], [2.0 ** -6], [0.0]]), b1=np.array([9.0, 9.0, 0.0]),
             W2=np.array([[1.0, 0, 0], [0, 1.0, 0], [0, 1.0, 0]]), b2=np.array([0.0, 3 * 2.0 ** -7, 2.0 ** -7]),
             W3=np.array([[1.0 + 2.0 ** -9, 2.0, 4.0]]), b3=np.array([0.5]))
    return MLP64(p), np.array([[1.0 + 2.0 ** -10]], np.float32)


def test_forward_bf16_rounding_points_by_hand():
    net, F = _tiny_net_for_rounding_points()
    assert net.forward_bf16(F)[0] == 63.5
    # the FP64 forward keeps every value: y = (1 + 2^-9) z0 + 2 (z1 + 3*2^-7) + 4 (z1 + 2^-7) + 0.5
    x = 1.0 + 2.0 ** -10
    z0, z1 = 9.0 + 2.0 ** -5 * x, 9.0 + 2.0 ** -6 * x
    want = (1 + 2.0 ** -9) * z0 + 2 * (z1 + 3 * 2.0 ** -7) + 4 * (z1 + 2.0 ** -7) + 0.5
    assert abs(net.forward(F)[0] - want) <= 1e-12


def test_forward_bf16_within_rounding_bound_of_forward():
    # Every BF16 rounding (to 8 significant bits) changes a value by at most
    # u = 2^-8 of it, and GELU is Lipschitz with constant L = Phi(sqrt2) + sqrt2 phi(sqrt2)
    # < 1.13.  Propagating: with x^ = x + dx, W^ = W + dW (|dW| <= u|W|):
    #   |z^ - z| <= |W| |dx| + u |W| |x^| + u |b|
    #   |h^ - h| <= L |z^ - z| + u |GELU(z^)|
    # layer by layer, then |y^ - y| <= |W3| |dh2| + u |W3| |h2^| + u |b3|.
    # The bound holds for every row; a dropped bias or layer, a transposed
    # weight or a rounding at the wrong place exceeds it on random nets.
    from oracle.mlp import MLP64, init_params, gelu
    u, L = 2.0 ** -8, 1.13
    rng = np.random.default_rng(9)
    for seed in range(4):
        p = init_params(7, 16, seed=seed)
        for k in p:
            p[k] = (p[k] + 0.2 * rng.normal(size=p[k].shape)).astype(np.float32)
        mu = rng.normal(size=7).astype(np.float32)
        sd = (0.5 + rng.random(7)).astype(np.float32)
        net = MLP64(p, mu=mu, sigma=sd)
        F = (rng.normal(size=(300, 7)) * sd + mu).astype(np.float32)
        y = net.forward(F)
        yb = net.forward_bf16(F)
        P = {k: np.abs(np.asarray(v, np.float64)) for k, v in net.p.items()}
        x = net.standardise(F)
        dx = np.abs(x) * (u + 2.0 ** -23) + 2.0 ** -23        # FP32 standardisation, then BF16
        xh = np.abs(x) + dx
        dz1 = dx @ P["W1"].T + u * xh @ P["W1"].T + u * P["b1"]
        z1 = x @ net.p["W1"].T + net.p["b1"]
        dh1 = L * dz1 + u * (np.abs(gelu(z1)) + L * dz1) + 2.0 ** -23 * (np.abs(gelu(z1)) + L * dz1)
        h1h = np.abs(gelu(z1)) + dh1
        dz2 = dh1 @ P["W2"].T + u * h1h @ P["W2"].T + u * P["b2"]
        z2 = gelu(z1) @ net.p["W2"].T + net.p["b2"]
        dh2 = L * dz2 + u * (np.abs(gelu(z2)) + L * dz2) + 2.0 ** -23 * (np.abs(gelu(z2)) + L * dz2)
        h2h = np.abs(gelu(z2)) + dh2
        dy = (dh2 @ P["W3"].T + u * h2h @ P["W3"].T + u * P["b3"])[:, 0]
        assert (np.abs(yb - y) <= dy * (1 + 1e-9)).all(), seed
        # and the rounding is not a no-op: the two differ on most rows
        assert (yb != y).mean() > 0.9
