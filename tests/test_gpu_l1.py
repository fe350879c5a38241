"""SuCo-L1 (Sec. 5.3, Table 5) on the GPU against the oracle's L1 forms,
through the C ABI (needs an MI355X): the k-medians build, the query path
stage by stage, exact search at alpha = beta = 1, byte rows, SC-Linear, the
Multi-sequence rule, persistence and the calls that stay Euclidean."""
import numpy as np
import pytest

import oracle
import synth
from parity import check_query, check_topk

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
    out = {}
    for key, v in o.items():
        if v is None:
            continue
        out[key] = v.view(torch.int16).cpu().numpy().view(np.uint16) if v.dtype == torch.uint16 else v.cpu().numpy()
    if "cand" in out:
        out["cand"] = np.sort(out["cand"], axis=1)
    return out


def make_l1(suco, X, ns, sk, iters=8, seed=1, flags=0):
    _, c32, asg, _ = oracle.build_index(X, ns, sk, iters=iters, seed=seed, metric=1)
    oix = oracle.Index(X, ns, sk, c32, asg, metric=1)
    gix = suco.Index.from_index(torch.from_numpy(X).cuda(), ns, sk, c32, asg, flags=suco.BUILD_L1 | flags)
    return oix, gix


@pytest.mark.parametrize("workload,n,ns,sk", [(2, 30_000, 8, 20), (1, 10_000, 8, 16)])
def test_l1_gpu_build_equals_oracle_kmedians(suco, workload, n, ns, sk):
    """The GPU's k-medians (L1 assignment in FP64, lower-median update by radix
    select) gives the oracle's centres and assignments bit for bit, on integer
    (SIFT-like) and real-valued (mixture) data."""
    W = synth.Workload(workload)
    X = W.data(n)
    print(f"case: l1 build workload={workload} n={n}", flush=True)
    _, c32, asg, _ = oracle.build_index(X, ns, sk, iters=5, seed=3, metric=1)
    gix = suco.Index.build(torch.from_numpy(X).cuda(), ns, sk, iters=5, seed=3, flags=suco.BUILD_L1)
    gc, ga = gix.export()
    assert np.array_equal(ga, asg)
    assert np.array_equal(gc, c32)
    assert gix.flags() & suco.INDEX_L1
    gix.free()


def test_l1_mixture_stage_parity(suco):
    """Every query compared with the oracle's SuCo-L1 stage by stage: cells
    (within the FP32/FP64 key band), SC-scores, candidates, top-k by L1."""
    W = synth.Workload(1)
    X, Q = W.data(), W.queries()
    print("case: l1 mixture128 n=10000 stage parity", flush=True)
    oix, gix = make_l1(suco, X, 8, 16)
    o = gix.query_debug(torch.from_numpy(Q).cuda(), 10, 0.05, 0.005)
    torch.cuda.synchronize()
    st = check_query(oix, X, Q, 10, 0.05, 0.005, to_np(o))
    assert st["band_queries"] <= 5
    gix.free()


@pytest.mark.parametrize("alpha", [0.003, 0.03])
def test_l1_sift_like_stage_parity(suco, alpha):
    """Integer data, n = 200,000: both activation paths and the sparse step."""
    W = synth.Workload(2)
    X, Q = W.data(200_000), W.queries(40)
    print(f"case: l1 sift_like n=200000 alpha={alpha}", flush=True)
    oix, gix = make_l1(suco, X, 8, 50, iters=4)
    o = gix.query_debug(torch.from_numpy(Q).cuda(), 10, alpha, 0.005)
    torch.cuda.synchronize()
    st = check_query(oix, X, Q, 10, alpha, 0.005, to_np(o))
    assert st["band_queries"] <= 3
    gix.free()


def test_l1_alpha_beta_one_is_exact_l1_search(suco):
    X = synth.tiny(2000, 24, 5, "int", levels=6)       # ties broken by id
    Q = synth.tiny(12, 24, 6, "int", levels=6)
    oix, gix = make_l1(suco, X, 4, 6)
    ids, dists = gix.query(torch.from_numpy(Q).cuda(), 16, 1.0, 1.0)
    torch.cuda.synchronize()
    e_ids, e_d = oracle.bruteforce(X, Q, 16, metric=1)
    assert np.array_equal(ids.cpu().numpy(), e_ids)
    assert np.array_equal(dists.cpu().numpy(), e_d.astype(np.float32))
    gix.free()


def test_l1_byte_rows_equal_fp32_rows(suco):
    """Integer rows: the re-rank from the byte copy gives the FP32 rows' L1
    results bitwise (every partial sum is an exact integer)."""
    W = synth.Workload(2)
    X, Q = W.data(50_000), W.queries(64)
    _, gix = make_l1(suco, X, 8, 20, iters=3)
    _, fix = make_l1(suco, X, 8, 20, iters=3, flags=suco.BUILD_NO_BYTE_ROWS)
    assert gix.flags() & suco.INDEX_BYTE_ROWS and not fix.flags() & suco.INDEX_BYTE_ROWS
    Qd = torch.from_numpy(Q).cuda()
    a = gix.query(Qd, 10, 0.01, 0.005)
    b = fix.query(Qd, 10, 0.01, 0.005)
    torch.cuda.synchronize()
    assert np.array_equal(a[0].cpu().numpy(), b[0].cpu().numpy())
    assert np.array_equal(a[1].cpu().numpy(), b[1].cpu().numpy())
    gix.free()
    fix.free()


def test_l1_sclinear_integer_bit_exact(suco):
    W = synth.Workload(2)
    X, Q = W.data(20_000), W.queries(30)
    _, gix = make_l1(suco, X, 8, 8, iters=2)
    print("case: l1 sclinear n=20000", flush=True)
    ids, d, sc = gix.query_sclinear(torch.from_numpy(Q).cuda(), 10, 0.03, 0.003, scores=True)
    torch.cuda.synchronize()
    r_ids, r_d, r_sc = oracle.sclinear(X, 8, Q, 10, 0.03, 0.003, want_scores=True, metric=1)
    assert np.array_equal(sc.cpu().numpy(), r_sc)
    assert np.array_equal(ids.cpu().numpy(), r_ids)
    assert np.array_equal(d.cpu().numpy(), r_d.astype(np.float32))
    gix.free()


def test_l1_multiseq_and_batched_equal_plain(suco):
    W = synth.Workload(2)
    X, Q = W.data(100_000), W.queries(300)
    _, gix = make_l1(suco, X, 8, 30, iters=3)
    Qd = torch.from_numpy(Q).cuda()
    a = gix.query(Qd, 10, 0.004, 0.005)
    gix.set_activation(suco.ACT_MULTISEQ)
    b = gix.query(Qd, 10, 0.004, 0.005)
    gix.set_activation(suco.ACT_DYNAMIC)
    bt = suco.Batcher(gix, 512, 10, 0.005)
    c_ids = torch.empty((300, 10), dtype=torch.int32, device="cuda")
    c_d = torch.empty((300, 10), dtype=torch.float32, device="cuda")
    bt.query(Qd[:200], alpha=0.004, out=(c_ids[:200], c_d[:200]))
    bt.query(Qd[200:], alpha=0.004, out=(c_ids[200:], c_d[200:]))
    torch.cuda.synchronize()
    for o in (b, (c_ids, c_d)):
        assert np.array_equal(a[0].cpu().numpy(), o[0].cpu().numpy())
        assert np.array_equal(a[1].cpu().numpy(), o[1].cpu().numpy())
    bt.free()
    gix.free()


def test_l1_save_load_and_euclidean_only_calls(suco, tmp_path):
    """The metric travels with a saved index; the learned budget and the
    split-precision build stay Euclidean (SUCO_E_UNSUPPORTED)."""
    X, Q = synth.Workload(1).data(), synth.Workload(1).queries(32)
    _, gix = make_l1(suco, X, 8, 16)
    path = str(tmp_path / "l1.suco")
    gix.save(path)
    lix = suco.Index.load(path, flags=0)          # the file's metric wins over the override
    assert lix.flags() & suco.INDEX_L1
    Qd = torch.from_numpy(Q).cuda()
    r0 = gix.query(Qd, 10, 0.05, 0.005)
    r1 = lix.query(Qd, 10, 0.05, 0.005)
    torch.cuda.synchronize()
    assert np.array_equal(r0[0].cpu().numpy(), r1[0].cpu().numpy())
    assert np.array_equal(r0[1].cpu().numpy(), r1[1].cpu().numpy())
    with pytest.raises(suco.SucoError) as e:
        suco.query_features(gix, Qd)
    assert e.value.code == suco.SUCO_E_UNSUPPORTED
    with pytest.raises(suco.SucoError) as e:
        suco.Index.build(torch.from_numpy(X).cuda(), 8, 16, iters=1, flags=suco.BUILD_L1 | suco.BUILD_BF16)
    assert e.value.code == suco.SUCO_E_UNSUPPORTED
    lix.free()
    gix.free()
