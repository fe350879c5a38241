"""SC-Linear on the GPU (Alg. 1) against the FP64 oracle's SC-Linear, through
the C ABI (needs an MI355X)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def suco():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_14754_amd as m
    m.lib()
    return m


def gpu_index(suco, X, ns, sk=4):
    _, c32, asg, _ = oracle.build_index(X, ns, sk, iters=2, seed=1)
    return suco.Index.from_index(torch.from_numpy(X).cuda(), ns, sk, c32, asg)


@pytest.mark.parametrize("alpha,beta,k", [(0.03, 0.003, 10), (0.01, 0.01, 50), (0.2, 0.002, 10)])
def test_sclinear_integer_data_bit_exact(suco, alpha, beta, k):
    """Integer coordinates: every subspace distance is an exact integer in FP32,
    so the GPU's SC-scores (Def. 4), candidates and top-k equal the oracle's."""
    W = synth.Workload(2)
    X, Q = W.data(20_000), W.queries(40)
    ix = gpu_index(suco, X, 8)
    print(f"case: sclinear sift_like n=20000 alpha={alpha} beta={beta} k={k}", flush=True)
    ids, d, sc = ix.query_sclinear(torch.from_numpy(Q).cuda(), k, alpha, beta, scores=True)
    torch.cuda.synchronize()
    r_ids, r_d, r_sc = oracle.sclinear(X, 8, Q, k, alpha, beta, want_scores=True)
    assert np.array_equal(sc.cpu().numpy(), r_sc)
    assert np.array_equal(ids.cpu().numpy(), r_ids)
    assert np.allclose(d.cpu().numpy(), r_d, rtol=1e-6, atol=1e-6)
    ix.free()


def test_sclinear_one_subspace_is_exact_knn(suco):
    """N_s = 1 (the subspace is the whole space) with A = B = k: the colliding
    points are the k nearest, so SC-Linear returns the exact k-NN (Def. 1)."""
    X = synth.tiny(5000, 32, 3, "int", levels=40)     # integer data: exact FP32 distances, id-ordered ties
    Q = synth.tiny(20, 32, 4, "int", levels=40)
    ix = gpu_index(suco, X, 1)
    k = 10
    ids, d, _ = ix.query_sclinear(torch.from_numpy(Q).cuda(), k, k / 5000, k / 5000)
    torch.cuda.synchronize()
    b_ids, b_d = oracle.bruteforce(X, Q, k)
    assert np.array_equal(ids.cpu().numpy(), b_ids)
    ix.free()


def test_sclinear_alpha_beta_one_is_exact_search(suco):
    X = synth.tiny(3000, 24, 5, "int", levels=9)      # many exact ties, all broken by id
    Q = synth.tiny(15, 24, 6, "int", levels=9)
    ix = gpu_index(suco, X, 4)
    ids, d, sc = ix.query_sclinear(torch.from_numpy(Q).cuda(), 7, 1.0, 1.0, scores=True)
    torch.cuda.synchronize()
    assert (sc.cpu().numpy() == 4).all()
    b_ids, b_d = oracle.bruteforce(X, Q, 7)
    assert np.array_equal(ids.cpu().numpy(), b_ids)
    ix.free()


def test_sclinear_real_data_within_the_tie_band(suco):
    """Real-valued data: the GPU ranks points in each subspace by FP32
    distances, the oracle by FP64; a point's score may differ only in
    subspaces where its FP64 distance is within 1e-5 (relative) of that
    subspace's A-th smallest, and then the GPU's candidates and top-k are the
    oracle's selection and re-rank applied to the GPU's scores."""
    W = synth.Workload(1)
    X, Q = W.data(), W.queries(30)
    ix = gpu_index(suco, X, 8)
    alpha, beta, k = 0.05, 0.005, 10
    ids, d, sc = ix.query_sclinear(torch.from_numpy(Q).cuda(), k, alpha, beta, scores=True)
    torch.cuda.synchronize()
    sc, ids, d = sc.cpu().numpy(), ids.cpu().numpy(), d.cpu().numpy()
    r_ids, r_d, r_sc = oracle.sclinear(X, 8, Q, k, alpha, beta, want_scores=True)
    n = X.shape[0]
    A, B = oracle.count_A(alpha, n), oracle.count_B(beta, n, k)
    dim0, w = oracle.layout(128, 8)
    X64 = X.astype(np.float64)
    for q in range(Q.shape[0]):
        diff = np.nonzero(sc[q] != r_sc[q])[0]
        if diff.size:
            near = np.zeros(diff.size, bool)
            for i in range(8):
                s0, sw = int(dim0[2 * i]), int(w[2 * i] + w[2 * i + 1])
                di = ((X64[:, s0:s0 + sw] - Q[q, s0:s0 + sw].astype(np.float64)) ** 2).sum(axis=1)
                kth = np.sort(di)[A - 1]
                near |= np.abs(di[diff] - kth) <= 1e-5 * kth
            assert near.all(), f"query {q}: scores differ away from a subspace threshold"
            assert (np.abs(sc[q][diff].astype(int) - r_sc[q][diff].astype(int)) <= 8).all()
        c = oracle.select(sc[q], B)
        e_ids, e_d = oracle.rerank(X, Q[q], c, k)
        assert np.array_equal(np.sort(ids[q]), np.sort(e_ids)) or np.allclose(d[q], e_d, rtol=1e-5)
    ix.free()
