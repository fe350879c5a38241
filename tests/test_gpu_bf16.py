"""BF16 split precision vs the plain path and the FP64 oracle, through the C ABI
(needs an MI355X).

 * Without BF16 centre distances the activation, collision and selection are
   the plain path's, and the certified survivor filter must keep the FP32
   top-k: ids and distances equal the plain query's bit for bit.
 * The MFMA centre distances are compared with the oracle's BF16 model (FP64
   distances of the BF16-rounded query halves and centres) within the FP32
   accumulation bound 2 (w + 4) 2^-24 (|q^| + |c^|)^2, w the half's width.
 * With BF16 centre distances the activated cells follow the oracle's BF16
   model except where keys tie within that bound (the band of the parity rule,
   widened by it), and everything after activation follows the usual rules.
"""
import numpy as np
import pytest

import oracle
import synth
from parity import check_query

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def suco():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_14754_amd as m
    m.lib()
    return m


def to_np(o):
    out = {}
    for key, v in o.items():
        if v is None:
            continue
        out[key] = v.view(torch.int16).cpu().numpy().view(np.uint16) if v.dtype == torch.uint16 else v.cpu().numpy()
    return out


def make(suco, X, ns, sk, iters=10, seed=1, **kw):
    _, c32, asg, _ = oracle.build_index(X, ns, sk, iters=iters, seed=seed)
    oix = oracle.Index(X, ns, sk, c32, asg)
    gix = suco.Index.from_index(torch.from_numpy(X).cuda(), ns, sk, c32, asg, flags=suco.BUILD_BF16, **kw)
    return oix, gix, c32


def half_bound(Q, c32, d, ns, sk):
    """[nq][2ns][sk] bound of |MFMA centre distance - BF16 model|, from the FP32 arithmetic."""
    dim0, wd = oracle.layout(d, ns)
    qb = oracle.bf16_round(Q).astype(np.float64)
    cb = oracle.bf16_round(c32).astype(np.float64)
    out = np.zeros((Q.shape[0], 2 * ns, sk))
    for g in range(2 * ns):
        d0, w = int(dim0[g]), int(wd[g])
        cen = cb[sk * d0: sk * d0 + sk * w].reshape(sk, w)
        nq_ = np.linalg.norm(qb[:, d0:d0 + w], axis=1)
        nc = np.linalg.norm(cen, axis=1)
        out[:, g, :] = 2 * (w + 4) * U32 * (nq_[:, None] + nc[None, :]) ** 2
    return out


def query_all(gix, Q, k, alpha, beta, **kw):
    o = gix.query_bf16(torch.from_numpy(Q).cuda(), k, alpha, beta, **kw)
    torch.cuda.synchronize()
    return to_np(o)


# ------------------------------------------------ certified survivors --
@pytest.mark.parametrize("k", [10, 1, 64])
def test_bf16_rerank_equals_plain_bitwise(suco, k):
    """Gaussian mixture n=10,000 d=128, N_s=8, sqrtK=16, 100 queries."""
    W = synth.Workload(1)
    X, Q = W.data(), W.queries()
    print(f"case: mixture128 bf16 re-rank k={k}", flush=True)
    oix, gix, _ = make(suco, X, 8, 16)
    assert gix.flags() & ~suco.INDEX_SPARSE == suco.INDEX_BF16   # real-valued data: no byte rows
    beta = 0.005 if k < 64 else 0.01
    ids, dists = gix.query(torch.from_numpy(Q).cuda(), k, 0.05, beta)
    b = query_all(gix, Q, k, 0.05, beta)
    assert np.array_equal(b["ids"], ids.cpu().numpy())
    assert np.array_equal(b["dists"], dists.cpu().numpy())
    B = oracle.count_B(beta, X.shape[0], k)
    assert (b["nsurv"] >= k).all() and (b["nsurv"] <= B).all()
    # the FP32 distance of each result against FP64: within the FP32 summation bound
    assert (b["relerr"] <= (X.shape[1] + 2) * U32).all()
    gix.free()


def test_bf16_survivors_keep_exact_ties(suco):
    """Integer rows with every point duplicated: many candidates tie exactly in
    distance; the survivors must keep all tied members so that ties resolve by id
    as in the plain path."""
    W = synth.Workload(2)
    half = W.data(10_000)
    X = np.ascontiguousarray(np.repeat(half, 2, axis=0))
    Q = W.queries(60)
    print("case: duplicated integer rows n=20000 d=128", flush=True)
    oix, gix, _ = make(suco, X, 8, 16)
    for k in (1, 9, 10, 33):
        ids, dists = gix.query(torch.from_numpy(Q).cuda(), k, 0.05, 0.01)
        b = query_all(gix, Q, k, 0.05, 0.01)
        assert np.array_equal(b["ids"], ids.cpu().numpy()), k
        assert np.array_equal(b["dists"], dists.cpu().numpy()), k
    ref = oix.query(Q, 10, 0.05, 0.01)
    b = query_all(gix, Q, 10, 0.05, 0.01)
    assert np.array_equal(b["ids"], ref["ids"])           # integer distances are exact on both sides
    gix.free()


def test_bf16_ragged_chunks_and_errors(suco):
    W = synth.Workload(1)
    X, Q = W.data(3000), W.queries(77)
    oix, gix, _ = make(suco, X, 4, 8, query_chunk=16)
    ids, dists = gix.query(torch.from_numpy(Q).cuda(), 10, 0.1, 0.02)
    b = query_all(gix, Q, 10, 0.1, 0.02)
    assert np.array_equal(b["ids"], ids.cpu().numpy()) and np.array_equal(b["dists"], dists.cpu().numpy())
    # empty batch, bad flags, index without BF16 data
    e = gix.query_bf16(torch.zeros((0, X.shape[1]), device="cuda"), 10, 0.1, 0.02)
    assert e["ids"].shape == (0, 10)
    with pytest.raises(suco.SucoError) as ei:
        suco.lib()
        import ctypes as C
        qd = torch.from_numpy(Q).cuda()
        out_i = torch.empty((77, 10), dtype=torch.int32, device="cuda")
        out_d = torch.empty((77, 10), dtype=torch.float32, device="cuda")
        suco._check(suco.lib().suco_query_bf16(gix._h, C.c_void_p(qd.data_ptr()), 77, 10, 0.1, 0.02, 6,
                                               C.c_void_p(out_i.data_ptr()), C.c_void_p(out_d.data_ptr()),
                                               None, None, None, None))
    assert ei.value.code == suco.SUCO_E_INVAL
    _, c32, asg, _ = oracle.build_index(X, 4, 8, iters=3)
    plain = suco.Index.from_index(torch.from_numpy(X).cuda(), 4, 8, c32, asg)
    with pytest.raises(suco.SucoError) as ei:
        plain.query_bf16(torch.from_numpy(Q).cuda(), 10, 0.1, 0.02)
    assert ei.value.code == suco.SUCO_E_STATE
    plain.free()
    gix.free()


def test_bf16_build_rejects_d_not_multiple_of_8(suco):
    X = synth.tiny(500, 12, 1, "gauss", levels=4)
    with pytest.raises(suco.SucoError) as ei:
        suco.Index.build(torch.from_numpy(X).cuda(), 2, 4, flags=suco.BUILD_BF16)
    assert ei.value.code == suco.SUCO_E_UNSUPPORTED


# ------------------------------------------------- MFMA centre distances --
@pytest.mark.parametrize("case", [
    ("mixture128", 1, 10_000, 8, 16, 37),     # halves of width 8, 16 centres
    ("gist_like", 3, 20_000, 20, 50, 40),     # width 24 (a ragged second k-step), 50 centres
    ("mixture128", 1, 10_000, 3, 128, 19),    # widths 21/22, the largest sqrtK, ragged query tile
])
def test_mfma_centre_distances_match_bf16_model(suco, case):
    name, c, n, ns, sk, nq = case
    W = synth.Workload(c)
    X, Q = W.data(n) if c != 3 else W._draw(synth._rng(4242, 0), n), W.queries(nq)
    print(f"case: centre distances {name} n={n} ns={ns} sk={sk} nq={nq}", flush=True)
    oix, gix, c32 = make(suco, X, ns, sk, iters=4)
    oix.set_s1_bf16(True)
    b = query_all(gix, Q, 10, 0.05, 0.005, s1_bf16=True, cdist=True)
    ref = np.zeros((nq, 2 * ns, sk))
    for q in range(nq):
        for g in range(2 * ns):
            ref[q, g] = oix.centroid_dists(Q[q], g)
    bound = half_bound(Q, c32, X.shape[1], ns, sk)
    err = np.abs(b["cdist"].astype(np.float64) - ref)
    assert (err <= bound).all(), float((err / bound).max())
    gix.free()


# ------------------------------------------- parity with the BF16 model --
def test_bf16_s1_parity_with_oracle_model(suco):
    """mixture128 with BF16 centre distances: the oracle with its BF16 step-1
    model, compared stage by stage under the widened band."""
    W = synth.Workload(1)
    X, Q = W.data(), W.queries()
    oix, gix, c32 = make(suco, X, 8, 16, iters=25)
    oix.set_s1_bf16(True)
    g = query_all(gix, Q, 10, 0.05, 0.005, s1_bf16=True, debug=True)
    hb = half_bound(Q, c32, X.shape[1], 8, 16)
    # a key is a sum over the two halves of a subspace; two keys can swap only
    # within the sum of both errors
    tol = np.zeros((Q.shape[0], 8))
    for i in range(8):
        tol[:, i] = 2 * (hb[:, 2 * i].max(axis=1) + hb[:, 2 * i + 1].max(axis=1))
    st = check_query(oix, X, Q, 10, 0.05, 0.005, g, key_tol=tol)
    assert st["band_queries"] <= 10
    assert st["agree"] >= 0.99
    assert (g["relerr"] <= (X.shape[1] + 2) * U32).all()
    gix.free()


# ------------------------------------------------------------ full size --
@pytest.mark.timeout(900)
def test_gist_like_full_size_sampled(suco):
    """GIST-like n=1,000,000 d=960 in (0,1), N_s=20, sqrtK=50, 1,000 queries,
    k=10, alpha=0.05, beta=0.005, BF16 centre distances and re-rank first pass
    (the benchmark's launch configuration); 8 sampled queries against the oracle's
    BF16 model, every query against the plain path's re-rank of its candidates."""
    W = synth.Workload(3)
    print("case: gist_like n=1e6 generating", flush=True)
    X, Q = W.data(), W.queries()
    print("case: gist_like oracle build", flush=True)
    _, c32, asg, _ = oracle.build_index(X, 20, 50, iters=2, seed=1)
    oix = oracle.Index(X, 20, 50, c32, asg)
    oix.set_s1_bf16(True)
    gix = suco.Index.from_index(torch.from_numpy(X).cuda(), 20, 50, c32, asg, flags=suco.BUILD_BF16)
    print("case: gist_like GPU bf16 query, full batch", flush=True)
    Qd = torch.from_numpy(Q).cuda()
    full = to_np(gix.query_bf16(Qd, 10, 0.05, 0.005, s1_bf16=True))
    # the certified filter: the plain FP32 re-rank of the same candidates gives the same answer
    print("case: gist_like plain re-rank of the bf16 candidates", flush=True)
    dbg = to_np(gix.query_bf16(Qd, 10, 0.05, 0.005, s1_bf16=True, debug=True, nsurv=False, relerr=False))
    assert np.array_equal(dbg["ids"], full["ids"]) and np.array_equal(dbg["dists"], full["dists"])
    ids32, d32 = gix.rerank(Qd, torch.from_numpy(dbg["cand"]).cuda(), 10)
    torch.cuda.synchronize()
    assert np.array_equal(full["ids"], ids32.cpu().numpy())
    assert np.array_equal(full["dists"], d32.cpu().numpy())
    assert (full["nsurv"] >= 10).all()
    assert (full["relerr"] <= (960 + 2) * U32).all()
    print(f"case: gist_like survivors mean {full['nsurv'].mean():.1f} max {full['nsurv'].max()}", flush=True)
    sample = np.sort(np.random.default_rng(0).choice(Q.shape[0], 8, replace=False))
    print("case: gist_like oracle on the sample", flush=True)
    gs = {key: v[sample] for key, v in dbg.items() if key in ("ids", "dists", "cand", "ncells", "aprime", "cells")}
    gs["scores"] = to_np(gix.query_bf16(Qd[sample].contiguous(), 10, 0.05, 0.005, s1_bf16=True,
                                        debug=True))["scores"]
    hb = half_bound(Q[sample], c32, 960, 20, 50)
    tol = np.zeros((len(sample), 20))
    for i in range(20):
        tol[:, i] = 2 * (hb[:, 2 * i].max(axis=1) + hb[:, 2 * i + 1].max(axis=1))
    st = check_query(oix, X, Q[sample], 10, 0.05, 0.005, gs, key_tol=tol)
    assert st["band_queries"] <= 4
    gix.free()
