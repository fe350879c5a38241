"""suco_query_noalloc (the entry point that allocates nothing) against
suco_query, through the C ABI (needs an MI355X)."""
import numpy as np
import pytest

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


def test_noalloc_equals_query_on_two_calls(suco):
    """Two calls in a row, the second smaller: bitwise the results of
    suco_query.  The first batch (5,000 queries at n = 10,000) needs two passes
    through the fixed scratch; the second call reuses the scratch the first
    left behind."""
    W = synth.Workload(1)
    X = torch.from_numpy(W.data()).cuda()
    ix = suco.Index.build(X, 8, 16, iters=6)
    Q1 = torch.from_numpy(W.queries(5000)).cuda()
    Q2 = torch.from_numpy(W.train_queries(37)).cuda()
    for Q, alpha, beta, k in ((Q1, 0.05, 0.005, 10), (Q2, 0.02, 0.01, 7)):
        print(f"case: noalloc nq={Q.shape[0]} alpha={alpha} beta={beta} k={k}", flush=True)
        a_ids, a_d = ix.query_noalloc(Q, k, alpha, beta)
        b_ids, b_d = ix.query(Q, k, alpha, beta)
        torch.cuda.synchronize()
        assert np.array_equal(a_ids.cpu().numpy(), b_ids.cpu().numpy())
        assert np.array_equal(a_d.cpu().numpy(), b_d.cpu().numpy())
    ix.free()


def test_noalloc_integer_rows_and_limits(suco):
    """SIFT-like integer rows (the byte re-rank path), then a shape whose one
    query needs more workspace than the scratch holds: SUCO_E_UNSUPPORTED
    before any work, and the next call still answers."""
    W = synth.Workload(2)
    X = torch.from_numpy(W.data(200_000)).cuda()
    ix = suco.Index.build(X, 8, 32, iters=4)
    Q = torch.from_numpy(W.queries(300)).cuda()
    print("case: noalloc sift_like n=200000 nq=300", flush=True)
    a = ix.query_noalloc(Q, 10, 0.01, 0.005)
    b = ix.query(Q, 10, 0.01, 0.005)
    torch.cuda.synchronize()
    assert np.array_equal(a[0].cpu().numpy(), b[0].cpu().numpy())
    assert np.array_equal(a[1].cpu().numpy(), b[1].cpu().numpy())
    n_big = 12_000_000
    print(f"case: noalloc limit n={n_big} beta=1", flush=True)
    Xb = torch.rand((n_big, 4), device="cuda")
    big = suco.Index.build(Xb, 2, 2, iters=1)
    del Xb
    with pytest.raises(suco.SucoError) as e:
        big.query_noalloc(Q[:2, :4].contiguous(), 5, 0.5, 1.0)
    assert e.value.code == suco.SUCO_E_UNSUPPORTED and "scratch" in str(e.value)
    big.free()
    Q2 = Q[:50].contiguous()
    a = ix.query_noalloc(Q2, 10, 0.01, 0.005)
    b = ix.query(Q2, 10, 0.01, 0.005)
    torch.cuda.synchronize()
    assert np.array_equal(a[0].cpu().numpy(), b[0].cpu().numpy())
    ix.free()
