"""Multi-sequence against Dynamic Activation on the GPU (Sec. 4.2): both rules
activate the same cells, so every later step gives the same result; the
Multi-sequence traversal takes its cells in ascending key order and matches
the oracle's cells within the FP32/FP64 tie band (needs an MI355X)."""
import numpy as np
import pytest

import oracle
import synth
from parity import REL, check_query, oracle_cells

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
    return out


@pytest.fixture(scope="module")
def sift200k(suco):
    W = synth.Workload(2)
    X, Q = W.data(200_000), W.queries(200)
    _, c32, asg, _ = oracle.build_index(X, 8, 50, iters=6, seed=1)
    oix = oracle.Index(X, 8, 50, c32, asg)
    gix = suco.Index.from_index(torch.from_numpy(X).cuda(), 8, 50, c32, asg)
    yield dict(X=X, Q=Q, oix=oix, gix=gix)
    gix.free()


def run(gix, form, Q, k, alpha, beta, alpha_q=None):
    import paper_2411_14754_amd as m
    gix.set_activation(form)
    aq = torch.from_numpy(alpha_q).cuda() if alpha_q is not None else None
    o = gix.query_debug(torch.from_numpy(Q).cuda(), k, alpha, beta, alpha_q=aq)
    torch.cuda.synchronize()
    gix.set_activation(m.ACT_DYNAMIC)
    return to_np(o)


def same_cells(a, b):
    assert np.array_equal(a["ncells"], b["ncells"])
    assert np.array_equal(a["aprime"], b["aprime"])
    nq, ns, _ = a["cells"].shape
    for q in range(nq):
        for i in range(ns):
            nc = a["ncells"][q, i]
            assert np.array_equal(np.sort(a["cells"][q, i, :nc]), np.sort(b["cells"][q, i, :nc])), (q, i)


@pytest.mark.parametrize("alpha", [0.0005, 0.003, 0.01, 0.05])
def test_multiseq_equals_dynamic_activation(suco, sift200k, alpha):
    """Same activated cells per (query, subspace) (as sets: Dynamic Activation
    writes them row by row), hence bitwise equal scores, candidates and top-k.
    alpha=0.0005 and 0.003 take Alg. 3's walk on the Dynamic Activation side,
    0.01 and 0.05 its bisection."""
    Q, gix = sift200k["Q"], sift200k["gix"]
    print(f"case: multiseq vs DA sift_like n=200000 alpha={alpha}", flush=True)
    da = run(gix, suco.ACT_DYNAMIC, Q, 10, alpha, 0.005)
    ms = run(gix, suco.ACT_MULTISEQ, Q, 10, alpha, 0.005)
    same_cells(da, ms)
    for key in ("scores", "ids", "dists", "feat"):
        assert np.array_equal(da[key], ms[key]), key
    assert np.array_equal(np.sort(da["cand"], axis=1), np.sort(ms["cand"], axis=1))


def test_multiseq_per_query_alpha(suco, sift200k):
    Q, gix = sift200k["Q"], sift200k["gix"]
    aq = np.exp(np.random.default_rng(3).uniform(np.log(1e-4), np.log(0.2), Q.shape[0])).astype(np.float32)
    print("case: multiseq vs DA sift_like n=200000 per-query alpha in [1e-4, 0.2]", flush=True)
    da = run(gix, suco.ACT_DYNAMIC, Q, 10, 0.0, 0.005, alpha_q=aq)
    ms = run(gix, suco.ACT_MULTISEQ, Q, 10, 0.0, 0.005, alpha_q=aq)
    same_cells(da, ms)
    assert np.array_equal(da["ids"], ms["ids"]) and np.array_equal(da["scores"], ms["scores"])


def test_multiseq_retrieval_order_and_oracle(suco, sift200k):
    """The Multi-sequence cells of 24 queries against the oracle's Multi-sequence
    form: equal sets (up to the tie band) and the GPU's retrieval order
    ascending in the oracle's FP64 keys (up to the band's tolerance); then the
    whole query against the oracle."""
    X, Q, oix, gix = sift200k["X"], sift200k["Q"][:24], sift200k["oix"], sift200k["gix"]
    alpha, beta = 0.01, 0.005
    print("case: multiseq vs oracle sift_like n=200000 alpha=0.01", flush=True)
    ms = run(gix, suco.ACT_MULTISEQ, Q, 10, alpha, beta)
    rc = oracle_cells(oix, Q, alpha, form=2)
    for q in range(Q.shape[0]):
        for i in range(oix.ns):
            _, _, key, _ = rc[q][i]
            g = ms["cells"][q, i, :ms["ncells"][q, i]].astype(np.int64)
            kg = key[g]
            assert (np.diff(kg) >= -REL * kg[1:]).all(), (q, i)
    st = check_query(oix, X, Q, 10, alpha, beta, ms)
    assert st["band_queries"] <= 2


def test_multiseq_limits(suco):
    """An index with sqrt_k above 64 has no Multi-sequence traversal; an unknown
    rule is an invalid argument."""
    import paper_2411_14754_amd as m
    X = synth.tiny(30_000, 16, 2)
    _, c32, asg, _ = oracle.build_index(X, 1, 80, iters=2, seed=1)
    gix = suco.Index.from_index(torch.from_numpy(X).cuda(), 1, 80, c32, asg)
    with pytest.raises(m.SucoError) as e:
        gix.set_activation(m.ACT_MULTISEQ)
    assert e.value.code == m.SUCO_E_UNSUPPORTED
    with pytest.raises(m.SucoError) as e:
        gix.set_activation(7)
    assert e.value.code == m.SUCO_E_INVAL
    gix.free()
