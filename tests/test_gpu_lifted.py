"""The lifted workload at full size (n = 10,000,000, d = 256, N_s = 16,
sqrtK = 64, beta = 0.003) with per-query alphas over the learned budget's
range: the GPU-built index's centres and assignments given to the oracle,
then 12 sampled queries of a 2,000-query call compared stage by stage (needs
an MI355X and ~25 GB of host memory)."""
import numpy as np
import pytest

import oracle
import synth
from parity import check_query

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def suco():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    psutil = pytest.importorskip("psutil")
    if psutil.virtual_memory().available < 40 * 2**30:
        pytest.skip("needs ~40 GB of free host memory")
    import paper_2411_14754_amd as m
    m.lib()
    return m


def test_lifted_full_size_sampled_parity(suco):
    W = synth.Workload(5)
    sp = W.spec
    n, d, ns, sk = sp["n"], sp["d"], sp["n_s"], sp["sqrt_k"]
    print(f"case: lifted256 n={n} d={d} generating", flush=True)
    X = W.data()
    Q = W.queries(2000)
    print("case: lifted256 GPU build (6 iterations)", flush=True)
    gix = suco.Index.build(torch.from_numpy(X).cuda(), ns, sk, iters=6, seed=1)
    c32, asg = gix.export()
    assert asg.shape == (2 * ns, n) and asg.min() >= 0 and asg.max() < sk
    oix = oracle.Index(X, ns, sk, c32, asg)
    del asg
    # per-query alphas log-uniform over the learned budget's range on this workload
    aq = np.exp(np.random.default_rng(5).uniform(np.log(1e-5), np.log(1e-3), 2000)).astype(np.float32)
    print("case: lifted256 2,000 queries in one call, per-query alpha in [1e-5, 1e-3]", flush=True)
    o = gix.query_debug(torch.from_numpy(Q).cuda(), 10, 0.0, sp["beta"], alpha_q=torch.from_numpy(aq).cuda(),
                        scores=False, cells=False)
    torch.cuda.synchronize()
    full = {k: v.cpu().numpy() for k, v in o.items() if v is not None}
    del o
    A = np.array([oracle.count_A(float(a), n) for a in aq])
    assert (full["aprime"] >= A[:, None]).all()
    sample = np.sort(np.random.default_rng(6).choice(2000, 12, replace=False))
    g = gix.query_debug(torch.from_numpy(Q[sample]).cuda(), 10, 0.0, sp["beta"],
                        alpha_q=torch.from_numpy(aq[sample]).cuda())
    torch.cuda.synchronize()
    gs = {}
    for key, v in g.items():
        if v is None:
            continue
        gs[key] = v.view(torch.int16).cpu().numpy().view(np.uint16) if v.dtype == torch.uint16 else v.cpu().numpy()
    gs["cand"] = np.sort(gs["cand"], axis=1)
    for key in ("ids", "dists", "ncells", "aprime"):
        assert np.array_equal(full[key][sample], gs[key]), key       # the sample answers as in the full call
    print("case: lifted256 oracle on 12 sampled queries", flush=True)
    st = check_query(oix, X, Q[sample], 10, aq[sample].astype(np.float64), sp["beta"], gs)
    assert st["band_queries"] <= 2
    gix.free()
