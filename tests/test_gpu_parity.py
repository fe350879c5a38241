"""GPU path vs the FP64 oracle, through the C ABI (needs an MI355X)."""
import numpy as np
import pytest

import oracle
import synth
from parity import cells_to_gpu_layout, check_query, check_topk, oracle_cells

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def suco():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_14754_amd as m
    m.lib()
    return m


def to_np(o):
    """Exported stages as NumPy arrays; candidate rows sorted (their order is unspecified)."""
    out = {}
    for key, v in o.items():
        if v is None:
            continue
        if v.dtype == torch.uint16:
            out[key] = v.view(torch.int16).cpu().numpy().view(np.uint16)
        else:
            out[key] = v.cpu().numpy()
    if "cand" in out:
        out["cand"] = np.sort(out["cand"], axis=1)
    return out


def debug(ix, Q, k, alpha, beta, alpha_q=None):
    Qd = torch.from_numpy(Q).cuda()
    aq = torch.from_numpy(alpha_q).cuda() if alpha_q is not None else None
    o = ix.query_debug(Qd, k, alpha, beta, alpha_q=aq)
    torch.cuda.synchronize()
    return to_np(o)


def make(X, ns, sk, iters=10, seed=1, **kw):
    import paper_2411_14754_amd as m
    _, c32, asg, _ = oracle.build_index(X, ns, sk, iters=iters, seed=seed)
    oix = oracle.Index(X, ns, sk, c32, asg)
    gix = m.Index.from_index(torch.from_numpy(X).cuda(), ns, sk, c32, asg, **kw)
    return oix, gix


# ------------------------------------------------------------- workloads --
def test_mixture128_full_parity(suco):
    """Gaussian mixture n=10,000 d=128, N_s=8, sqrtK=16, 100 queries, k=10,
    alpha=0.05, beta=0.005: every query compared stage by stage."""
    W = synth.Workload(1)
    X, Q = W.data(), W.queries()
    print("case: mixture128 n=10000 d=128 ns=8 sk=16 nq=100", flush=True)
    oix, gix = make(X, 8, 16, iters=25)
    g = debug(gix, Q, 10, 0.05, 0.005)
    st = check_query(oix, X, Q, 10, 0.05, 0.005, g)
    assert st["band_queries"] <= 5
    assert st["agree"] >= 0.999
    gix.free()


def test_stage_collide_select_from_oracle_cells(suco):
    """Steps 3-4 fed with the oracle's activated cells: bit-exact scores and candidates."""
    W = synth.Workload(1)
    X, Q = W.data(), W.queries(40)
    oix, gix = make(X, 8, 16)
    # the last case has fewer colliding points than B, so score-0 points are selected too (T = 0)
    for alpha, beta, k in ((0.05, 0.005, 10), (0.2, 0.01, 10), (0.01, 0.001, 5), (1.0, 0.003, 10), (1e-4, 0.1, 10)):
        rc = oracle_cells(oix, Q, alpha)
        cells, nc = cells_to_gpu_layout([[r[0] for r in row] for row in rc], Q.shape[0], 8, 256)
        ref = oix.query(Q, k, alpha, beta, want_scores=True, want_cand=True)
        cand, sc = gix.collide_select(torch.from_numpy(cells.view(np.int16)).cuda().view(torch.uint16),
                                      torch.from_numpy(nc).cuda(), k, beta)
        torch.cuda.synchronize()
        assert np.array_equal(sc.cpu().numpy(), ref["scores"]), (alpha, beta)
        cand = np.sort(cand.cpu().numpy(), axis=1)
        assert (np.diff(cand, axis=1) > 0).all()                       # B distinct ids
        assert np.array_equal(cand, np.sort(ref["cand"], axis=1)), (alpha, beta)
    gix.free()


def test_stage_rerank_from_oracle_candidates(suco):
    W = synth.Workload(1)
    X, Q = W.data(), W.queries(50)
    oix, gix = make(X, 8, 16)
    for beta, k in ((0.005, 10), (0.05, 64), (0.0001, 1), (1.0, 10)):
        ref = oix.query(Q, k, 0.05, beta, want_cand=True)
        ids, dists = gix.rerank(torch.from_numpy(Q).cuda(), torch.from_numpy(ref["cand"]).cuda(), k)
        torch.cuda.synchronize()
        check_topk(X, Q, ids.cpu().numpy(), dists.cpu().numpy(), ref["ids"], ref["dists"], k)
    gix.free()


def test_integer_data_rerank_is_exact(suco):
    """SIFT-like integer data: FP32 distances are exact integers, so ids and
    distances equal the oracle's exactly (ties broken by id on both sides)."""
    W = synth.Workload(2)
    X, Q = W.data(20_000), W.queries(30)
    oix, gix = make(X, 8, 16)
    ref = oix.query(Q, 10, 0.05, 0.01, want_cand=True)
    ids, dists = gix.rerank(torch.from_numpy(Q).cuda(), torch.from_numpy(ref["cand"]).cuda(), 10)
    torch.cuda.synchronize()
    assert np.array_equal(ids.cpu().numpy(), ref["ids"])
    assert np.array_equal(dists.cpu().numpy().astype(np.float64), ref["dists"].astype(np.float32).astype(np.float64))
    gix.free()


def test_gpu_build_equals_oracle_build(suco):
    """Create Index on the GPU (FP64 k-means, IMI) gives the oracle's centres and assignments."""
    W = synth.Workload(1)
    X = W.data(6000)
    c64, c32, asg, _ = oracle.build_index(X, 8, 16, iters=12, seed=7)
    gix = suco.Index.build(torch.from_numpy(X).cuda(), 8, 16, iters=12, seed=7)
    gc, ga = gix.export()
    assert np.array_equal(ga, asg)
    assert np.array_equal(gc, c32)
    # and the GPU-built index answers like the oracle's index
    oix = oracle.Index(X, 8, 16, c32, asg)
    Q = W.queries(20)
    g = debug(gix, Q, 10, 0.05, 0.01)
    check_query(oix, X, Q, 10, 0.05, 0.01, g)
    gix.free()


def test_gpu_build_integer_data(suco):
    W = synth.Workload(2)
    X = W.data(30_000)
    _, c32, asg, _ = oracle.build_index(X, 8, 20, iters=6, seed=3)
    gix = suco.Index.build(torch.from_numpy(X).cuda(), 8, 20, iters=6, seed=3)
    gc, ga = gix.export()
    assert np.array_equal(ga, asg) and np.array_equal(gc, c32)
    gix.free()


# ------------------------------------------------------------ edge cases --
def test_alpha_beta_one_is_exact_search(suco):
    X = synth.tiny(2000, 24, 5, "clustered")
    Q = synth.tiny(12, 24, 6, "clustered")
    oix, gix = make(X, 4, 6)
    ids, dists = gix.query(torch.from_numpy(Q).cuda(), 16, 1.0, 1.0)
    torch.cuda.synchronize()
    e_ids, e_d = oracle.bruteforce(X, Q, 16)
    check_topk(X, Q, ids.cpu().numpy(), dists.cpu().numpy(), e_ids, e_d, 16)
    gix.free()


def test_ragged_tiles_and_chunks(suco):
    """n not a multiple of the tile, several tiles, queries split in ragged chunks;
    results bitwise equal across chunkings."""
    X = synth.tiny(3001, 32, 8, "clustered")
    Q = synth.tiny(30, 32, 9, "clustered")
    oix, gix = make(X, 4, 6, tile_max=512, query_chunk=7)
    g = debug(gix, Q, 8, 0.1, 0.02)
    check_query(oix, X, Q, 8, 0.1, 0.02, g)
    _, c32, asg, _ = oracle.build_index(X, 4, 6, iters=10)
    g2ix = suco.Index.from_index(torch.from_numpy(X).cuda(), 4, 6, c32, asg, query_chunk=1000)
    g2 = debug(g2ix, Q, 8, 0.1, 0.02)
    for key in ("ids", "dists", "scores", "cand", "ncells", "aprime"):
        assert np.array_equal(g[key], g2[key]), key
    gix.free()
    g2ix.free()


def test_single_cell_index(suco):
    X = synth.tiny(700, 16, 10, "gauss")
    Q = synth.tiny(5, 16, 11, "gauss")
    oix, gix = make(X, 4, 1)
    g = debug(gix, Q, 5, 0.05, 0.02)
    assert (g["scores"] == 4).all()
    assert np.array_equal(g["cand"], np.tile(np.arange(14), (5, 1)))
    check_query(oix, X, Q, 5, 0.05, 0.02, g)
    gix.free()


@pytest.mark.parametrize("k", [1, 64])
def test_k_extremes(suco, k):
    W = synth.Workload(1)
    X, Q = W.data(5000), W.queries(10)
    oix, gix = make(X, 8, 8)
    g = debug(gix, Q, k, 0.1, 0.02)
    check_query(oix, X, Q, k, 0.1, 0.02, g)
    gix.free()


@pytest.mark.parametrize("alpha", [0.01, 0.05])
def test_sqrt_k_above_64(suco, alpha):
    """sqrtK = 100 (the activation step's 128-thread form): activated cells,
    scores, candidates and top-k against the oracle, at a small and a large budget."""
    W = synth.Workload(1)
    X, Q = W.data(30_000), W.queries(20)
    print(f"case: sqrtK=100 n=30000 alpha={alpha}", flush=True)
    oix, gix = make(X, 4, 100, iters=4)
    g = debug(gix, Q, 10, alpha, 0.01)
    assert g["ncells"].sum() > g["ncells"].size        # several cells somewhere
    st = check_query(oix, X, Q, 10, alpha, 0.01, g)
    assert st["band_queries"] <= 2
    gix.free()


@pytest.mark.parametrize("alpha,beta", [(0.0005, 0.005), (0.003, 0.005), (0.01, 0.005), (0.05, 0.002),
                                        (0.3, 0.01), (0.0001, 0.2), (0.0002, 0.4)])
def test_sparse_step_equals_tiled_step(suco, alpha, beta):
    """The sparse collision step (SC-scores per bucket of 4096 ids, one or
    several LDS rounds) against the tiled step on the same index: candidates,
    SC-scores and top-k bitwise.  The budgets span one round, several rounds,
    queries left to the tiled step (too many points), T = 0 (fewer than B
    colliding points: the lowest score-0 ids fill the candidates, in the
    sparse step when B <= 65,536, else in the tiled one), all in one batch
    with per-query alphas around alpha."""
    W = synth.Workload(2)
    X = W.data(200_000)
    Q = W.queries(300)
    _, c32, asg, _ = oracle.build_index(X, 8, 32, iters=3, seed=2)
    Xd = torch.from_numpy(X).cuda()
    sp = suco.Index.from_index(Xd, 8, 32, c32, asg)
    td = suco.Index.from_index(Xd, 8, 32, c32, asg, flags=suco.BUILD_NO_SPARSE)
    aq = (alpha * np.exp(np.random.default_rng(1).uniform(-1.0, 1.0, Q.shape[0]))).astype(np.float32)
    aq = np.minimum(aq, 1.0).astype(np.float32)
    print(f"case: sparse vs tiled alpha~{alpha} beta={beta}", flush=True)
    a = debug(sp, Q, 10, 0.0, beta, alpha_q=aq)
    b = debug(td, Q, 10, 0.0, beta, alpha_q=aq)
    for key in ("ids", "dists", "cand", "scores", "ncells", "aprime"):
        assert np.array_equal(a[key], b[key]), key
    sp.profile(True)
    sp.query_alpha(torch.from_numpy(Q).cuda(), 10, torch.from_numpy(aq).cuda(), beta)
    prof = sp.profile_read()
    print("profile", {k: v for k, v in prof.items() if v[1]}, flush=True)
    sp.free()
    td.free()


@pytest.mark.parametrize("ns,alpha,beta", [(16, 0.003, 0.005), (16, 0.0005, 0.02), (20, 0.01, 0.005),
                                           (31, 0.002, 0.01)])
def test_sparse_step_five_bit_scores(suco, ns, alpha, beta):
    """N_s of 16 to 31: the sparse step keeps 5-bit scores (six ids a window
    word) and equals the tiled step bitwise: candidates, SC-scores, top-k."""
    W = synth.Workload(2)
    X = W.data(100_000)
    Q = W.queries(200)
    _, c32, asg, _ = oracle.build_index(X, ns, 16, iters=2, seed=3)
    Xd = torch.from_numpy(X).cuda()
    sp = suco.Index.from_index(Xd, ns, 16, c32, asg)
    td = suco.Index.from_index(Xd, ns, 16, c32, asg, flags=suco.BUILD_NO_SPARSE)
    assert sp.flags() & suco.INDEX_SPARSE and not td.flags() & suco.INDEX_SPARSE
    aq = (alpha * np.exp(np.random.default_rng(2).uniform(-1.0, 1.0, Q.shape[0]))).astype(np.float32)
    print(f"case: five-bit sparse vs tiled ns={ns} alpha~{alpha} beta={beta}", flush=True)
    a = debug(sp, Q, 10, 0.0, beta, alpha_q=aq)
    b = debug(td, Q, 10, 0.0, beta, alpha_q=aq)
    for key in ("ids", "dists", "cand", "scores", "ncells", "aprime"):
        assert np.array_equal(a[key], b[key]), key
    # the sparse step took the queries: the tiled collision step had little left to do
    Qd, aqd = torch.from_numpy(Q).cuda(), torch.from_numpy(aq).cuda()
    prof = {}
    for name, ix in (("sparse", sp), ("tiled", td)):
        ix.profile(True)
        ix.profile_read()
        ix.query_alpha(Qd, 10, aqd, beta)
        prof[name] = ix.profile_read()
        ix.profile(False)
    assert prof["sparse"]["collide"][0] < 0.5 * prof["tiled"]["collide"][0]
    sp.free()
    td.free()


def test_per_query_alpha(suco):
    W = synth.Workload(1)
    X, Q = W.data(8000), W.queries(25)
    oix, gix = make(X, 8, 12)
    aq = np.random.default_rng(0).uniform(0.005, 0.3, size=25).astype(np.float32)
    g = debug(gix, Q, 10, 0.0, 0.01, alpha_q=aq)
    check_query(oix, X, Q, 10, aq.astype(np.float64), 0.01, g)
    gix.free()


def test_per_query_alpha_outside_the_unit_interval(suco):
    """Device alphas are not checked on the host: above 1, +inf and NaN give the
    results of alpha = 1, and values <= 0 those of one activated point."""
    W = synth.Workload(1)
    X, Q = W.data(6000), W.queries(6)
    _, gix = make(X, 8, 12)
    Qd = torch.from_numpy(Q).cuda()
    odd = np.array([np.nan, np.inf, 2.0, 0.0, -1.0, -np.inf], np.float32)
    ids, d = gix.query_alpha(Qd, 10, torch.from_numpy(odd).cuda(), 0.01)
    top, _ = gix.query(Qd, 10, 1.0, 0.01)
    one, _ = gix.query(Qd, 10, 1.0 / 6000, 0.01)
    torch.cuda.synchronize()
    ids, top, one = ids.cpu().numpy(), top.cpu().numpy(), one.cpu().numpy()
    assert np.array_equal(ids[:3], top[:3])
    assert np.array_equal(ids[3:], one[3:])
    gix.free()


def test_save_load_round_trip(suco, tmp_path):
    """suco_index_save / suco_index_load: the loaded index exports the saved
    centres and assignments (the oracle's, for an imported index), keeps its
    flags, and answers every query bitwise as the saved one; a corrupted file
    is refused by its checksum."""
    W = synth.Workload(1)
    X, Q = W.data(), W.queries(64)
    oix, gix = make(X, 8, 16, iters=8)
    Qd = torch.from_numpy(Q).cuda()
    path = str(tmp_path / "mix.suco")
    gix.save(path)
    lix = suco.Index.load(path)
    assert (lix.n, lix.d, lix.ns, lix.sqrt_k) == (gix.n, gix.d, gix.ns, gix.sqrt_k)
    c0, a0 = gix.export()
    c1, a1 = lix.export()
    assert np.array_equal(c0.view(np.uint32), c1.view(np.uint32)) and np.array_equal(a0, a1)
    assert np.array_equal(c1, oix.cent32) and np.array_equal(a1, oix.assign)
    assert lix.flags() == gix.flags()
    r0 = gix.query(Qd, 10, 0.05, 0.005)
    r1 = lix.query(Qd, 10, 0.05, 0.005)
    torch.cuda.synchronize()
    assert np.array_equal(r0[0].cpu().numpy(), r1[0].cpu().numpy())
    assert np.array_equal(r0[1].cpu().numpy(), r1[1].cpu().numpy())
    lix.free()
    # a GPU-built BF16 index on integer data keeps its byte rows and BF16 copy
    Xi = synth.Workload(2).data(20_000)
    bix = suco.Index.build(torch.from_numpy(Xi).cuda(), 8, 10, iters=3, flags=suco.BUILD_BF16)
    bpath = str(tmp_path / "bf16.suco")
    bix.save(bpath)
    blix = suco.Index.load(bpath)
    assert blix.flags() == bix.flags() == suco.INDEX_BYTE_ROWS | suco.INDEX_BF16 | suco.INDEX_SPARSE
    Qi = torch.from_numpy(synth.Workload(2).queries(32)).cuda()
    s0 = bix.query_bf16(Qi, 10, 0.02, 0.01)
    s1 = blix.query_bf16(Qi, 10, 0.02, 0.01)
    torch.cuda.synchronize()
    assert np.array_equal(s0["ids"].cpu().numpy(), s1["ids"].cpu().numpy())
    assert np.array_equal(s0["dists"].cpu().numpy(), s1["dists"].cpu().numpy())
    bix.free()
    blix.free()
    # one flipped byte in the data section
    raw = bytearray(open(path, "rb").read())
    raw[-100] ^= 0x40
    bad = str(tmp_path / "bad.suco")
    open(bad, "wb").write(bytes(raw))
    with pytest.raises(suco.SucoError) as e:
        suco.Index.load(bad)
    assert e.value.code == suco.SUCO_E_INVAL and "checksum" in str(e.value)
    gix.free()


def test_empty_batch_and_errors(suco):
    W = synth.Workload(1)
    X = W.data(1000)
    _, gix = make(X, 8, 4)
    Q0 = torch.zeros((0, 128), device="cuda")
    ids, d = gix.query(Q0, 5, 0.1, 0.1)
    assert ids.shape == (0, 5)
    Q = torch.zeros((2, 128), device="cuda")
    with pytest.raises(suco.SucoError) as e:
        gix.query(Q, 65, 0.1, 0.1)                  # valid k, past the kernels' top-k lists
    assert e.value.code == suco.SUCO_E_UNSUPPORTED
    with pytest.raises(suco.SucoError) as e:
        gix.query(Q, 1001, 0.1, 0.1)                # k > n
    assert e.value.code == suco.SUCO_E_INVAL
    with pytest.raises(suco.SucoError):
        gix.query(Q, 5, 0.0, 0.1)
    with pytest.raises(suco.SucoError):
        gix.query(Q, 5, 0.1, 1.5)
    gix.free()
    with pytest.raises(suco.SucoError):
        suco.Index.build(torch.zeros((10, 8), device="cuda"), 5, 2)      # n_s > d/2
    with pytest.raises(suco.SucoError):
        suco.Index.build(torch.zeros((10, 8), device="cuda"), 2, 11)     # sqrt_k > n


def test_deterministic_repeat(suco):
    W = synth.Workload(1)
    X, Q = W.data(), W.queries(64)
    _, gix = make(X, 8, 16)
    a = debug(gix, Q, 10, 0.05, 0.005)
    b = debug(gix, Q, 10, 0.05, 0.005)
    for key in a:
        assert np.array_equal(a[key], b[key]), key
    gix.free()


def test_tie_level_left_out_of_later_tiles(suco):
    """Many tiles and a tie at level 1 (fewer than B points score 2 or more):
    the collision step leaves the level-1 ids of later tiles out of its lists
    once the block's earlier tiles hold B of them.  2,048 queries in one pass
    take one block per query (every tile seen in order); a sample of 24 takes
    several blocks per query.  Both give the oracle's candidates."""
    W = synth.Workload(2)
    X, Q = W.data(200_000), W.queries(2048)
    _, c32, asg, _ = oracle.build_index(X, 8, 50, iters=4, seed=1)
    oix = oracle.Index(X, 8, 50, c32, asg)
    gix = suco.Index.from_index(torch.from_numpy(X).cuda(), 8, 50, c32, asg, tile_max=4096)
    alpha, beta = 0.003, 0.005
    o = gix.query_debug(torch.from_numpy(Q).cuda(), 10, alpha, beta, scores=False, cells=False)
    torch.cuda.synchronize()
    full = to_np(o)
    del o
    sample = np.sort(np.random.default_rng(1).choice(Q.shape[0], 24, replace=False))
    gs = debug(gix, Q[sample], 10, alpha, beta)
    for key in ("ids", "dists", "cand"):
        assert np.array_equal(full[key][sample], gs[key]), key
    B = oracle.count_B(beta, X.shape[0], 10)
    ge2 = (gs["scores"] >= 2).sum(axis=1)
    assert (ge2 < B).all()                                  # the threshold is 1 for the sample
    st = check_query(oix, X, Q[sample], 10, alpha, beta, gs)
    assert st["band_queries"] <= 3
    gix.free()


# ----------------------------------------------------------- full size --
@pytest.fixture(scope="module")
def sift1m(suco):
    """SIFT-like n=1,000,000 d=128 (integers 0..255), N_s=8, sqrtK=50: the
    oracle's index, the same index on the GPU, 10,000 queries, and the exact
    top-50 of the first 512 queries (FP64 products, exact for these integers)."""
    W = synth.Workload(2)
    print("case: sift_like n=1e6 generating", flush=True)
    X, Q = W.data(), W.queries()
    print("case: sift_like oracle build", flush=True)
    _, c32, asg, _ = oracle.build_index(X, 8, 50, iters=6, seed=1)
    oix = oracle.Index(X, 8, 50, c32, asg)
    gix = suco.Index.from_index(torch.from_numpy(X).cuda(), 8, 50, c32, asg)
    del asg
    print("case: sift_like exact top-50 of 512 queries", flush=True)
    X64 = X.astype(np.float64)
    xx = (X64 * X64).sum(axis=1)
    gt = np.zeros((512, 50), np.int64)
    for q0 in range(0, 512, 64):
        q = Q[q0:q0 + 64].astype(np.float64)
        d2 = xx[None, :] - 2.0 * (q @ X64.T) + (q * q).sum(axis=1)[:, None]
        part = np.argpartition(d2, 100, axis=1)[:, :101]
        for r in range(q.shape[0]):
            cand = part[r][np.lexsort((part[r], d2[r, part[r]]))]
            assert d2[r, cand[49]] < d2[r, cand[100]]     # no tie crosses the shortlist's end
            gt[q0 + r] = cand[:50]
    del X64
    yield dict(X=X, Q=Q, oix=oix, gix=gix, gt=gt)
    gix.free()


def _full_and_sample(gix, Q, k, alpha, beta, alpha_q=None, seed=0):
    Qd = torch.from_numpy(Q).cuda()
    aq = torch.from_numpy(alpha_q).cuda() if alpha_q is not None else None
    o = gix.query_debug(Qd, k, alpha, beta, alpha_q=aq, scores=False, cells=False)
    torch.cuda.synchronize()
    full = to_np(o)
    del o
    sample = np.sort(np.random.default_rng(seed).choice(Q.shape[0], 24, replace=False))
    gs = debug(gix, Q[sample], k, alpha, beta, alpha_q=None if alpha_q is None else alpha_q[sample])
    for key in ("ids", "dists", "cand", "ncells", "aprime", "feat"):
        assert np.array_equal(full[key][sample], gs[key]), key        # batching does not change results
    return full, sample, gs


def _full_batch_properties(full, n, k, alpha, beta):
    B = oracle.count_B(beta, n, k)
    A = np.array([oracle.count_A(float(a), n) for a in np.ravel(alpha)])
    assert (full["aprime"] >= (A if A.size == 1 else A[:, None])).all()
    assert (np.diff(full["cand"], axis=1) > 0).all() and full["cand"].shape[1] == B
    assert ((full["cand"] >= 0) & (full["cand"] < n)).all()


def test_sift_like_full_size_sampled(suco, sift1m):
    """10,000 queries in one call at alpha=0.03 (the bisection path of the
    activation step); 24 sampled queries compared with the oracle stage by stage."""
    X, Q, oix, gix = sift1m["X"], sift1m["Q"], sift1m["oix"], sift1m["gix"]
    print("case: sift_like alpha=0.03 full batch and sample", flush=True)
    full, sample, gs = _full_and_sample(gix, Q, 10, 0.03, 0.005)
    print("case: sift_like alpha=0.03 oracle on the sample", flush=True)
    st = check_query(oix, X, Q[sample], 10, 0.03, 0.005, gs)
    assert st["band_queries"] <= 3
    assert (gs["scores"].sum(axis=1, dtype=np.int64) == gs["aprime"].sum(axis=1)).all()
    _full_batch_properties(full, X.shape[0], 10, 0.03, 0.005)


def _recall(ids, gt, k):
    return float(np.mean([len(set(a[:k].tolist()) & set(b[:k].tolist())) / k for a, b in zip(ids, gt)]))


def test_sift_like_operating_point(suco, sift1m):
    """The benchmark's operating point: alpha=0.003 (Alg. 3's walk in the
    activation step), beta=0.005, k=10, 10,000 queries in one call.  24 sampled
    queries stage by stage; over the first 512 queries the GPU's recall@10 is
    within 0.001 of the oracle's (both against the exact top-10)."""
    X, Q, oix, gix, gt = sift1m["X"], sift1m["Q"], sift1m["oix"], sift1m["gix"], sift1m["gt"]
    print("case: sift_like alpha=0.003 full batch and sample", flush=True)
    full, sample, gs = _full_and_sample(gix, Q, 10, 0.003, 0.005, seed=1)
    print("case: sift_like alpha=0.003 oracle on the sample", flush=True)
    st = check_query(oix, X, Q[sample], 10, 0.003, 0.005, gs)
    assert st["band_queries"] <= 3
    _full_batch_properties(full, X.shape[0], 10, 0.003, 0.005)
    print("case: sift_like alpha=0.003 oracle on 512 queries", flush=True)
    ref = oix.query(Q[:512], 10, 0.003, 0.005)
    r_gpu, r_ref = _recall(full["ids"][:512], gt, 10), _recall(ref["ids"], gt, 10)
    print(f"recall@10 GPU {r_gpu:.5f} oracle {r_ref:.5f}", flush=True)
    assert abs(r_gpu - r_ref) <= 0.001


def test_sift_like_learned_range_alphas(suco, sift1m):
    """Per-query alphas drawn log-uniformly in [0.0005, 0.01] (the range the
    learned budget uses; both activation paths occur), 10,000 queries in one
    call: 24 sampled queries stage by stage against the oracle on the same
    alphas, and the recall rule over the first 512 queries."""
    X, Q, oix, gix, gt = sift1m["X"], sift1m["Q"], sift1m["oix"], sift1m["gix"], sift1m["gt"]
    rng = np.random.default_rng(7)
    aq = np.exp(rng.uniform(np.log(0.0005), np.log(0.01), Q.shape[0])).astype(np.float32)
    print("case: sift_like per-query alpha full batch and sample", flush=True)
    full, sample, gs = _full_and_sample(gix, Q, 10, 0.0, 0.005, alpha_q=aq, seed=2)
    print("case: sift_like per-query alpha oracle on the sample", flush=True)
    st = check_query(oix, X, Q[sample], 10, aq[sample].astype(np.float64), 0.005, gs)
    assert st["band_queries"] <= 3
    _full_batch_properties(full, X.shape[0], 10, aq.astype(np.float64), 0.005)
    ref = oix.query(Q[:512], 10, aq[:512].astype(np.float64), 0.005)
    r_gpu, r_ref = _recall(full["ids"][:512], gt, 10), _recall(ref["ids"], gt, 10)
    print(f"recall@10 GPU {r_gpu:.5f} oracle {r_ref:.5f}", flush=True)
    assert abs(r_gpu - r_ref) <= 0.001


def test_sift_like_k50(suco, sift1m):
    """k=50 (the other k of the SIFT-like workload) at alpha=0.01: sampled
    queries stage by stage and the recall@50 rule over the first 512 queries."""
    X, Q, oix, gix, gt = sift1m["X"], sift1m["Q"], sift1m["oix"], sift1m["gix"], sift1m["gt"]
    print("case: sift_like k=50 alpha=0.01 full batch and sample", flush=True)
    full, sample, gs = _full_and_sample(gix, Q, 50, 0.01, 0.005, seed=3)
    print("case: sift_like k=50 oracle on the sample", flush=True)
    st = check_query(oix, X, Q[sample], 50, 0.01, 0.005, gs)
    assert st["band_queries"] <= 3
    _full_batch_properties(full, X.shape[0], 50, 0.01, 0.005)
    ref = oix.query(Q[:512], 50, 0.01, 0.005)
    r_gpu, r_ref = _recall(full["ids"][:512], gt, 50), _recall(ref["ids"], gt, 50)
    print(f"recall@50 GPU {r_gpu:.5f} oracle {r_ref:.5f}", flush=True)
    assert abs(r_gpu - r_ref) <= 0.001


def test_sift_like_batcher_with_model(suco, sift1m):
    """A batcher with a network attached, fed the 10,000 queries as uneven
    batches (1..4096): bitwise equal to suco_query_alpha on the alphas the
    network gives, and a sample of those queries matches the oracle."""
    X, Q, oix, gix = sift1m["X"], sift1m["Q"], sift1m["oix"], sift1m["gix"]
    Qd = torch.from_numpy(Q).cuda()
    net = suco.MLP(17, seed=21)
    F = suco.query_features(gix, Qd)
    net.set_norm(F.mean(dim=0).cpu().numpy(), F.std(dim=0).cpu().numpy())
    amin, amax, scale = 0.0005, 0.01, 0.003
    print("case: sift_like batcher with model, uneven stream", flush=True)
    b = suco.Batcher(gix, 4096, 10, 0.005)
    b.set_model(net, scale, amin, amax)
    out_ids = torch.empty((Q.shape[0], 10), dtype=torch.int32, device="cuda")
    out_d = torch.empty((Q.shape[0], 10), dtype=torch.float32, device="cuda")
    start = 0
    for sz in synth.Workload(2).batch_sizes(Q.shape[0]):
        b.query(Qd[start:start + sz], out=(out_ids[start:start + sz], out_d[start:start + sz]))
        start += sz
    ids, d, au = suco.query_learned(gix, net, Qd, 10, 0.005, scale, amin, amax)
    p_ids, p_d = gix.query_alpha(Qd, 10, au, 0.005)
    torch.cuda.synchronize()
    b.free()
    assert np.array_equal(out_ids.cpu().numpy(), p_ids.cpu().numpy())
    assert np.array_equal(out_d.cpu().numpy(), p_d.cpu().numpy())
    assert np.array_equal(ids.cpu().numpy(), p_ids.cpu().numpy())
    aq = au.cpu().numpy()
    assert (aq >= amin).all() and (aq <= amax).all() and len(np.unique(aq)) > 100
    sample = np.sort(np.random.default_rng(4).choice(Q.shape[0], 12, replace=False))
    gs = debug(gix, Q[sample], 10, 0.0, 0.005, alpha_q=aq[sample])
    assert np.array_equal(gs["ids"], p_ids.cpu().numpy()[sample])
    print("case: sift_like batcher with model, oracle on the sample", flush=True)
    st = check_query(oix, X, Q[sample], 10, aq[sample].astype(np.float64), 0.005, gs)
    assert st["band_queries"] <= 2


def test_byte_rows_equal_fp32_rows(suco):
    """Integer data in 0..255: the re-rank from the index's byte copy of X gives
    bitwise the results of the FP32 rows (and the oracle's top-k exactly)."""
    W = synth.Workload(2)
    X, Q = W.data(50_000), W.queries(200)
    _, c32, asg, _ = oracle.build_index(X, 8, 20, iters=4)
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    a = suco.Index.from_index(Xd, 8, 20, c32, asg)
    b = suco.Index.from_index(Xd, 8, 20, c32, asg, flags=suco.BUILD_NO_BYTE_ROWS)
    assert a.flags() & ~suco.INDEX_SPARSE == suco.INDEX_BYTE_ROWS and b.flags() & ~suco.INDEX_SPARSE == 0
    ra = a.query(Qd, 10, 0.02, 0.01)
    rb = b.query(Qd, 10, 0.02, 0.01)
    torch.cuda.synchronize()
    assert np.array_equal(ra[0].cpu().numpy(), rb[0].cpu().numpy())
    assert np.array_equal(ra[1].cpu().numpy(), rb[1].cpu().numpy())
    oix = oracle.Index(X, 8, 20, c32, asg)
    ref = oix.query(Q, 10, 0.02, 0.01)
    assert np.array_equal(ra[0].cpu().numpy(), ref["ids"])
    # queries that are not all bytes (a fraction, a value above 255) take the
    # FP32 arithmetic on the byte rows, mixed in one batch with byte queries
    Qm = Q.copy()
    Qm[::2, 3] += 0.5
    Qm[1::4, 7] = 256.0
    Qmd = torch.from_numpy(Qm).cuda()
    ra = a.query(Qmd, 10, 0.02, 0.01)
    rb = b.query(Qmd, 10, 0.02, 0.01)
    torch.cuda.synchronize()
    assert np.array_equal(ra[0].cpu().numpy(), rb[0].cpu().numpy())
    assert np.array_equal(ra[1].cpu().numpy(), rb[1].cpu().numpy())
    ref = oix.query(Qm, 10, 0.02, 0.01)
    check_topk(X, Qm, ra[0].cpu().numpy(), ra[1].cpu().numpy(), ref["ids"], ref["dists"], 10)
    a.free()
    b.free()
