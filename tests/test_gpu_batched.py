"""Batched form (HIP graphs over persistent kernels): bitwise equal to the plain
path for every batch size, through the C ABI (needs an MI355X)."""
import os

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


@pytest.fixture(scope="module")
def mixture_index(suco):
    W = synth.Workload(1)
    X = W.data()
    _, c32, asg, _ = oracle.build_index(X, 8, 16, iters=10)
    ix = suco.Index.from_index(torch.from_numpy(X).cuda(), 8, 16, c32, asg)
    Q = torch.from_numpy(W.queries(4096)).cuda()
    yield ix, Q
    ix.free()


def plain(ix, Q, k, alpha, beta, alpha_q=None):
    if alpha_q is None:
        ids, d = ix.query(Q, k, alpha, beta)
    else:
        ids, d = ix.query_alpha(Q, k, alpha_q, beta)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), d.cpu().numpy()


@pytest.mark.parametrize("nq", [1, 2, 63, 64, 65, 100, 1000, 1025, 4095, 4096])
def test_batched_equals_plain(suco, mixture_index, nq):
    ix, Q = mixture_index
    print(f"case: batched nq={nq}", flush=True)
    b = suco.Batcher(ix, 4096, 10, 0.005)
    ids, d = b.query(Q[:nq], alpha=0.05)
    torch.cuda.synchronize()
    p_ids, p_d = plain(ix, Q[:nq], 10, 0.05, 0.005)
    assert np.array_equal(ids.cpu().numpy(), p_ids)
    assert np.array_equal(d.cpu().numpy().view(np.uint32), p_d.view(np.uint32))
    b.free()


def test_uneven_stream_and_reuse(suco, mixture_index):
    """A stream of random batch sizes reuses each bucket's graph; every batch matches."""
    ix, Q = mixture_index
    b = suco.Batcher(ix, 4096, 10, 0.005)
    sizes = synth.Workload(4).batch_sizes(12000, 4096)
    start = 0
    for s in sizes:
        lo = start % 4096
        s = min(s, 4096 - lo) or 1
        q = Q[lo:lo + s]
        ids, d = b.query(q, alpha=0.02)
        torch.cuda.synchronize()
        p_ids, p_d = plain(ix, q, 10, 0.02, 0.005)
        assert np.array_equal(ids.cpu().numpy(), p_ids), s
        assert np.array_equal(d.cpu().numpy(), p_d), s
        start += s
    b.free()


def test_per_query_alpha_batched(suco, mixture_index):
    ix, Q = mixture_index
    aq = torch.from_numpy(np.random.default_rng(1).uniform(0.01, 0.2, 700).astype(np.float32)).cuda()
    b = suco.Batcher(ix, 1024, 10, 0.01)
    ids, d = b.query(Q[:700], alpha_q=aq)
    torch.cuda.synchronize()
    p_ids, p_d = plain(ix, Q[:700], 10, 0.0, 0.01, alpha_q=aq)
    assert np.array_equal(ids.cpu().numpy(), p_ids)
    assert np.array_equal(d.cpu().numpy(), p_d)
    b.free()


def test_multi_batches_in_one_launch(suco, mixture_index):
    """Uneven batches (one of them empty) handed over in one call equal each
    batch through its own call, with one alpha and with per-query alphas."""
    ix, Q = mixture_index
    sizes = [37, 0, 1, 700, 129, 1000, 64]
    starts = np.cumsum([0] + sizes)
    parts = [Q[starts[j]:starts[j + 1]] for j in range(len(sizes))]
    aq = torch.from_numpy(np.random.default_rng(2).uniform(0.01, 0.2, int(starts[-1])).astype(np.float32)).cuda()
    aparts = [aq[starts[j]:starts[j + 1]] for j in range(len(sizes))]
    b = suco.Batcher(ix, 2048, 10, 0.005)
    for per_query in (False, True):
        print(f"case: multi per_query={per_query}", flush=True)
        outs = b.query_multi(parts, alpha=0.05, alpha_qs=aparts if per_query else None)
        torch.cuda.synchronize()
        for j, q in enumerate(parts):
            assert outs[j][0].shape == (sizes[j], 10)
            if sizes[j] == 0:
                continue
            ids, d = (b.query(q, alpha_q=aparts[j]) if per_query else b.query(q, alpha=0.05))
            torch.cuda.synchronize()
            assert np.array_equal(outs[j][0].cpu().numpy(), ids.cpu().numpy()), j
            assert np.array_equal(outs[j][1].cpu().numpy().view(np.uint32), d.cpu().numpy().view(np.uint32)), j
        p_ids, p_d = plain(ix, Q[:int(starts[-1])], 10, 0.05, 0.005, alpha_q=aq if per_query else None)
        assert np.array_equal(torch.cat([o[0] for o in outs]).cpu().numpy(), p_ids)
    # a second call with fewer, smaller batches reuses the buffers of the first
    outs = b.query_multi(parts[:2], alpha=0.05)
    torch.cuda.synchronize()
    assert np.array_equal(outs[0][0].cpu().numpy(), plain(ix, parts[0], 10, 0.05, 0.005)[0])
    b.free()


def test_multi_errors(suco, mixture_index):
    ix, Q = mixture_index
    b = suco.Batcher(ix, 256, 10, 0.005)
    with pytest.raises(suco.SucoError):
        b.query_multi([Q[:1]] * 17, alpha=0.05)                    # more than 16 batches
    with pytest.raises(suco.SucoError):
        b.query_multi([Q[:200], Q[:100]], alpha=0.05)              # total beyond max_batch
    with pytest.raises(suco.SucoError):
        b.query_multi([Q[:10]], alpha=0.0)
    outs = b.query_multi([Q[:0], Q[:0]], alpha=0.05)
    assert outs[0][0].shape == (0, 10)
    b.free()


def test_tune_file_round_trip(suco, mixture_index, tmp_path):
    ix, Q = mixture_index
    path = str(tmp_path / "tune.txt")
    b1 = suco.Batcher(ix, 512, 10, 0.005, tune_file=path)
    r1 = b1.query(Q[:300], alpha=0.05)
    torch.cuda.synchronize()
    t1 = b1.tuning(512)
    assert os.path.exists(path) and "bucket=512" in open(path).read()
    b2 = suco.Batcher(ix, 512, 10, 0.005, tune_file=path)
    r2 = b2.query(Q[:300], alpha=0.05)
    torch.cuda.synchronize()
    t2 = b2.tuning(512)
    assert {k: v for k, v in t1.items() if k != "ms"} == {k: v for k, v in t2.items() if k != "ms"}
    assert np.array_equal(r1[0].cpu().numpy(), r2[0].cpu().numpy())
    b1.free()
    b2.free()


def test_batcher_errors(suco, mixture_index):
    ix, Q = mixture_index
    b = suco.Batcher(ix, 100, 10, 0.005)
    with pytest.raises(suco.SucoError):
        b.query(Q[:200], alpha=0.05)          # beyond max_batch (rounded up to 128)
    with pytest.raises(suco.SucoError):
        b.query(Q[:10], alpha=0.0)
    ids, _ = b.query(Q[:0], alpha=0.05)
    assert ids.shape == (0, 10)
    b.free()
    with pytest.raises(suco.SucoError):
        suco.Batcher(ix, 0, 10, 0.005)


def test_sift_like_uneven_stream_full_size(suco):
    """SIFT-like 1M x 128: 10,000 queries as uneven batches (1..4096) through the
    batcher equal the plain path's results for every query."""
    W = synth.Workload(2)
    X, Qn = W.data(), W.queries()
    Xd, Q = torch.from_numpy(X).cuda(), torch.from_numpy(Qn).cuda()
    print("case: sift_like batched: building", flush=True)
    ix = suco.Index.build(Xd, 8, 50, iters=4)
    p_ids, p_d = plain(ix, Q, 10, 0.003, 0.005)
    b = suco.Batcher(ix, 4096, 10, 0.005)
    out_ids = torch.empty((Q.shape[0], 10), dtype=torch.int32, device="cuda")
    out_d = torch.empty((Q.shape[0], 10), dtype=torch.float32, device="cuda")
    start = 0
    for s in W.batch_sizes(Q.shape[0]):
        b.query(Q[start:start + s], alpha=0.003, out=(out_ids[start:start + s], out_d[start:start + s]))
        start += s
    torch.cuda.synchronize()
    assert np.array_equal(out_ids.cpu().numpy(), p_ids)
    assert np.array_equal(out_d.cpu().numpy(), p_d)
    b.free()
    # the same uneven batches handed over together, in one launch
    b = suco.Batcher(ix, Q.shape[0], 10, 0.005)
    sizes = W.batch_sizes(Q.shape[0])
    starts = np.cumsum([0] + list(sizes))
    outs = [(out_ids[starts[j]:starts[j + 1]], out_d[starts[j]:starts[j + 1]]) for j in range(len(sizes))]
    out_ids.zero_()
    b.query_multi([Q[starts[j]:starts[j + 1]] for j in range(len(sizes))], alpha=0.003, outs=outs)
    torch.cuda.synchronize()
    assert np.array_equal(out_ids.cpu().numpy(), p_ids)
    assert np.array_equal(out_d.cpu().numpy(), p_d)
    b.free()
    ix.free()


@pytest.mark.timeout(900)
def test_deep_like_stream_full_size(suco):
    """Deep-like n=10,000,000 d=96 unit-norm rows, N_s=8, sqrtK=64, 100,000
    queries as uneven batches (1..4096), k=10, alpha=0.02, beta=0.002 (the
    batched workload at its real size): the stream equals the plain path for
    every query, and 4 sampled queries match the oracle stage by stage."""
    from parity import check_query
    W = synth.Workload(4)
    print("case: deep_like n=1e7 generating", flush=True)
    X, Qn = W.data(), W.queries()
    print("case: deep_like oracle build", flush=True)
    _, c32, asg, _ = oracle.build_index(X, 8, 64, iters=2, seed=1)
    oix = oracle.Index(X, 8, 64, c32, asg)
    Xd, Q = torch.from_numpy(X).cuda(), torch.from_numpy(Qn).cuda()
    ix = suco.Index.from_index(Xd, 8, 64, c32, asg)
    del asg
    print("case: deep_like plain, one call", flush=True)
    p_ids, p_d = plain(ix, Q, 10, 0.02, 0.002)
    print("case: deep_like batched stream", flush=True)
    b = suco.Batcher(ix, 4096, 10, 0.002)
    out_ids = torch.empty((Q.shape[0], 10), dtype=torch.int32, device="cuda")
    out_d = torch.empty((Q.shape[0], 10), dtype=torch.float32, device="cuda")
    start = 0
    for s in W.batch_sizes(Q.shape[0]):
        b.query(Q[start:start + s], alpha=0.02, out=(out_ids[start:start + s], out_d[start:start + s]))
        start += s
    torch.cuda.synchronize()
    assert np.array_equal(out_ids.cpu().numpy(), p_ids)
    assert np.array_equal(out_d.cpu().numpy(), p_d)
    b.free()
    sample = np.sort(np.random.default_rng(0).choice(Q.shape[0], 4, replace=False))
    print("case: deep_like GPU stages on the sample", flush=True)
    o = ix.query_debug(Q[sample].contiguous(), 10, 0.02, 0.002)
    torch.cuda.synchronize()
    gs = {key: (v.view(torch.int16).cpu().numpy().view(np.uint16) if v.dtype == torch.uint16 else v.cpu().numpy())
          for key, v in o.items() if v is not None}
    del o
    assert np.array_equal(gs["ids"], p_ids[sample])
    print("case: deep_like oracle on the sample", flush=True)
    st = check_query(oix, X, Qn[sample], 10, 0.02, 0.002, gs)
    assert st["band_queries"] <= 2
    ix.free()
