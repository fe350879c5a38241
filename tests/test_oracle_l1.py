"""CPU pins of the oracle's SuCo-L1 (Sec. 5.3, Table 5): Manhattan centre
distances, k-medians clustering, SC-Linear and SuCo under L1, each against a
closed form, a library routine, an invariant or brute force on tiny inputs."""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
import synth


def l1_knn(X, q, k):
    """Exact k-NN by (Manhattan distance, id) with SciPy's cityblock distance."""
    d = cdist(q[None, :].astype(np.float64), X.astype(np.float64), metric="cityblock")[0]
    order = np.lexsort((np.arange(X.shape[0]), d))[:k]
    return order, d[order]


def l1_index(n=600, d=16, ns=4, sk=4, seed=3, kind="clustered", iters=10):
    X = synth.tiny(n, d, seed, kind, levels=4)
    c64, c32, asg, obj = oracle.build_index(X, ns, sk, iters=iters, seed=seed, metric=1)
    return X, oracle.Index(X, ns, sk, c32, asg, metric=1), (c64, c32, asg, obj)


def test_l1_centre_distances_closed_form():
    """Query at the origin, centres at scaled unit vectors and a diagonal: the
    L1 distances are known integers (and the L2 index gives their squares)."""
    sk, w = 3, 4
    X = np.zeros((9, 2 * w), np.float32)
    asg = np.zeros((2, 9), np.int32)
    cent = np.zeros(sk * 2 * w, np.float32)
    half0 = np.array([[3, 0, 0, 0], [0, -5, 0, 0], [1, 1, 1, 1]], np.float32)
    cent[:sk * w] = half0.reshape(-1)
    cent[sk * w:] = (2 * half0).reshape(-1)
    q = np.zeros(2 * w, np.float32)
    ix1 = oracle.Index(X, 1, sk, cent, asg, metric=1)
    ix2 = oracle.Index(X, 1, sk, cent, asg, metric=0)
    assert np.array_equal(ix1.centroid_dists(q, 0), [3.0, 5.0, 4.0])
    assert np.array_equal(ix1.centroid_dists(q, 1), [6.0, 10.0, 8.0])
    assert np.array_equal(ix2.centroid_dists(q, 0), [9.0, 25.0, 4.0])


def test_kmedians_one_iteration_is_lower_median_of_members():
    """After one iteration every centre coordinate is the lower median (the
    ceil(m/2)-th smallest) of its members' values under the L1 assignment to
    the initial rows, and the final assignment is the L1 argmin (ties to the
    lowest id); the objectives are the L1 sums of those assignments."""
    X = synth.tiny(400, 6, 17, "int", levels=7)
    d0, w = oracle.layout(6, 1)
    init = oracle.init_ids(X, 1, 5, 2, 0)
    cent, asg, obj = oracle.kmeans(X, int(d0[0]), int(w[0]), 5, 1, init, metric=1)
    H = X[:, d0[0]:d0[0] + w[0]].astype(np.float64)
    c0 = H[init]
    D0 = cdist(H, c0, metric="cityblock")
    a0 = np.argmin(D0, axis=1)
    for c in range(5):
        mem = H[a0 == c]
        if len(mem) == 0:
            assert np.array_equal(cent[c], c0[c])
            continue
        lower = np.sort(mem, axis=0)[(len(mem) - 1) // 2]
        assert np.array_equal(cent[c], lower)
    D1 = cdist(H, cent, metric="cityblock")
    assert np.array_equal(asg, np.argmin(D1, axis=1))
    assert obj[0] == D0.min(axis=1).sum() and obj[1] == D1.min(axis=1).sum()


def test_kmedians_objective_non_increasing_and_medians_optimal():
    """Each k-medians step can only lower the sum of L1 distances; at the end
    every centre coordinate minimises its members' sum of absolute deviations
    (checked against every member value as an alternative)."""
    X = synth.tiny(700, 8, 23, "gauss")
    d0, w = oracle.layout(8, 1)
    init = oracle.init_ids(X, 1, 6, 4, 0)
    cent, asg, obj = oracle.kmeans(X, int(d0[0]), int(w[0]), 6, 12, init, metric=1)
    assert (np.diff(obj) <= 1e-9 * obj[0]).all()
    H = X[:, d0[0]:d0[0] + w[0]].astype(np.float64)
    # the centres were computed from the previous assignment; recompute it
    _, a_prev, _ = oracle.kmeans(X, int(d0[0]), int(w[0]), 6, 11, init, metric=1)
    for c in range(6):
        mem = H[a_prev == c]
        if len(mem) == 0:
            continue
        for j in range(w[0]):
            sad = np.abs(mem[:, j] - cent[c, j]).sum()
            alt = np.abs(mem[:, j][:, None] - mem[:, j][None, :]).sum(axis=0)
            assert sad <= alt.min() * (1 + 1e-12)


def test_kmedians_separates_obvious_clusters():
    rng = np.random.default_rng(4)
    centres = np.array([[-10.0, 0.0], [0.0, 10.0], [10.0, 0.0]])
    lab = rng.integers(0, 3, 600)
    X = (centres[lab] + 0.1 * rng.laplace(size=(600, 2))).astype(np.float32)
    init = np.array([np.flatnonzero(lab == c)[0] for c in (2, 0, 1)], np.int64)
    cent, a, _ = oracle.kmeans(X, 0, 2, 3, 20, init, metric=1)
    assert np.array_equal(a, np.array([1, 2, 0])[lab])
    assert np.allclose(cent, centres[[2, 0, 1]], atol=0.05)


def test_bruteforce_l1_matches_scipy():
    X = synth.tiny(300, 9, 5, "int", levels=5)          # many ties, broken by id
    Q = synth.tiny(6, 9, 6, "int", levels=5)
    ids, dist = oracle.bruteforce(X, Q, 12, metric=1)
    for qi, q in enumerate(Q):
        e_ids, e_d = l1_knn(X, q, 12)
        assert np.array_equal(ids[qi], e_ids)
        assert np.array_equal(dist[qi], e_d)


@pytest.mark.parametrize("kind", ["gauss", "int", "clustered"])
def test_l1_alpha_beta_one_is_exact_l1_search(kind):
    X, ix, _ = l1_index(kind=kind)
    Q = synth.tiny(6, 16, 98, kind, levels=4)
    out = ix.query(Q, 8, 1.0, 1.0)
    ids_l, _ = oracle.sclinear(X, 4, Q, 8, 1.0, 1.0, metric=1)
    for qi, q in enumerate(Q):
        e_ids, e_d = l1_knn(X, q, 8)
        assert np.array_equal(out["ids"][qi], e_ids)
        assert np.array_equal(ids_l[qi], e_ids)
        assert np.allclose(out["dists"][qi], e_d, rtol=1e-12)


def test_sclinear_l1_single_subspace_is_exact_knn():
    X = synth.tiny(500, 10, 7, "gauss")
    Q = synth.tiny(5, 10, 8, "gauss")
    ids, dist = oracle.sclinear(X, 1, Q, 7, 7 / 500, 7 / 500, metric=1)
    for qi, q in enumerate(Q):
        e_ids, e_d = l1_knn(X, q, 7)
        assert np.array_equal(ids[qi], e_ids)
        assert np.allclose(dist[qi], e_d, rtol=1e-12)


@pytest.mark.parametrize("seed,kind", [(1, "gauss"), (2, "int")])
def test_sclinear_l1_scores_equal_rank_count(seed, kind):
    """Def. 4 under L1: a point scores in subspace i when fewer than A points
    precede it in (L1 distance, id) order, by pairwise comparison."""
    X = synth.tiny(300, 12, seed, kind, levels=3)
    Q = synth.tiny(4, 12, seed + 100, kind, levels=3)
    ns, alpha = 3, 0.1
    A = oracle.count_A(alpha, 300)
    _, _, sc = oracle.sclinear(X, ns, Q, 5, alpha, 0.05, want_scores=True, metric=1)
    d0, w = oracle.layout(12, ns)
    for qi, q in enumerate(Q):
        expect = np.zeros(300, np.int64)
        for i in range(ns):
            lo, hi = d0[2 * i], d0[2 * i] + w[2 * i] + w[2 * i + 1]
            dsub = np.abs(X[:, lo:hi].astype(np.float64) - q[lo:hi]).sum(axis=1)
            less = (dsub[None, :] < dsub[:, None]) | ((dsub[None, :] == dsub[:, None]) &
                                                      (np.arange(300)[None, :] < np.arange(300)[:, None]))
            expect += less.sum(axis=1) < A
        assert np.array_equal(sc[qi].astype(np.int64), expect)


def test_l1_suco_scores_count_activated_cells():
    """SuCo-L1 with a budget below n: each point's score is the number of
    subspaces whose activated cells (the oracle's own, in L1 key order) hold
    it, and the activated cells are the shortest prefix of the cells sorted by
    L1 distance to their product centre (ties by ranks) that reaches A."""
    X, ix, (_, c32, asg, _) = l1_index(kind="gauss", seed=9)
    Q = synth.tiny(3, 16, 77, "gauss")
    alpha = 0.12
    out = ix.query(Q, 5, alpha, 0.05, want_scores=True)
    A = oracle.count_A(alpha, X.shape[0])
    d0, w = oracle.layout(16, 4)
    cent = c32.reshape(-1)
    for qi, q in enumerate(Q):
        expect = np.zeros(X.shape[0], np.int64)
        for i in range(4):
            g1, g2 = 2 * i, 2 * i + 1
            C1 = cent[4 * d0[g1]:4 * d0[g1] + 4 * w[g1]].reshape(4, w[g1]).astype(np.float64)
            C2 = cent[4 * d0[g2]:4 * d0[g2] + 4 * w[g2]].reshape(4, w[g2]).astype(np.float64)
            # L1 distance of q's subspace to every product centre, straight from its definition
            key = np.array([[np.abs(np.concatenate([C1[a], C2[b]]) -
                                    q[d0[g1]:d0[g1] + w[g1] + w[g2]].astype(np.float64)).sum()
                             for b in range(4)] for a in range(4)])
            # ranks of the centres of each half by (L1 distance, id): the tie order of the cells
            h1 = np.abs(C1 - q[d0[g1]:d0[g1] + w[g1]]).sum(axis=1)
            h2 = np.abs(C2 - q[d0[g2]:d0[g2] + w[g2]]).sum(axis=1)
            r1 = np.argsort(np.lexsort((np.arange(4), h1)))
            r2 = np.argsort(np.lexsort((np.arange(4), h2)))
            cells = sorted(((key[a, b], r1[a], r2[b], a * 4 + b) for a in range(4) for b in range(4)))
            taken, got = [], 0
            for _, _, _, c in cells:
                m = (asg[g1] == c // 4) & (asg[g2] == c % 4)
                taken.append(m)
                got += int(m.sum())
                if got >= A:
                    break
            expect += np.any(taken, axis=0)
        assert np.array_equal(out["scores"][qi].astype(np.int64), expect)
