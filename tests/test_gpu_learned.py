"""Learned activation budget on the GPU: gradients, training and inference
against the FP64 oracle, the learned query against the plain path, and the gain
of the trained network over a fixed alpha (needs an MI355X)."""
import numpy as np
import pytest

import oracle
import synth
from oracle.mlp import MLP64, PARAM_NAMES
from parity import check_query

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def suco():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_14754_amd as m
    m.lib()
    return m


def split(flat, n_in, H=128):
    shapes = dict(W1=(H, n_in), b1=(H,), W2=(H, H), b2=(H,), W3=(1, H), b3=(1,))
    out, o = {}, 0
    for k in PARAM_NAMES:
        sz = int(np.prod(shapes[k]))
        out[k] = flat[o:o + sz].reshape(shapes[k])
        o += sz
    return out


def test_gradients_match_oracle(suco):
    rng = np.random.default_rng(0)
    n_in, m = 17, 200
    net = suco.MLP(n_in, seed=3)
    flat = net.params().astype(np.float64)
    flat += 0.05 * rng.normal(size=flat.shape)            # non-zero biases too
    net.set_params(flat.astype(np.float32))
    mu = rng.normal(size=n_in).astype(np.float32)
    sd = (0.5 + rng.random(n_in)).astype(np.float32)
    net.set_norm(mu, sd)
    F = rng.normal(size=(m, n_in)).astype(np.float32) * sd + mu
    t = rng.normal(size=m).astype(np.float32)
    loss, g = net.forward_backward(torch.from_numpy(F).cuda(), torch.from_numpy(t).cuda())
    torch.cuda.synchronize()
    ref = MLP64(split(net.params().astype(np.float64), n_in), mu=mu, sigma=sd)
    r_loss, r_g = ref.loss_and_grad(F, t)
    assert abs(float(loss.item()) - r_loss) <= 1e-5 * max(1.0, r_loss)
    gg = split(g.cpu().numpy().astype(np.float64), n_in)
    for k in PARAM_NAMES:
        err = np.linalg.norm(gg[k] - r_g[k]) / max(1e-30, np.linalg.norm(r_g[k]))
        assert err <= 1e-4, (k, err)


def test_adam_step_matches_oracle(suco):
    rng = np.random.default_rng(1)
    n_in, m = 9, 128
    net = suco.MLP(n_in, seed=5)
    F = rng.normal(size=(m, n_in)).astype(np.float32)
    t = rng.normal(size=m).astype(np.float32)
    before = net.params().astype(np.float64)
    ref = MLP64(split(before, n_in))
    _, r_g = ref.loss_and_grad(F, t)
    ref.adam_step(r_g, {}, lr=1e-3)
    net.train_epoch(torch.from_numpy(F).cuda(), torch.from_numpy(t).cuda(), batch=m, lr=1e-3)
    after = split(net.params().astype(np.float64), n_in)
    for k in PARAM_NAMES:
        big = np.abs(r_g[k]) > 1e-6 * np.abs(r_g[k]).max()
        assert np.allclose(after[k][big], ref.p[k][big], atol=1e-6, rtol=1e-6), k


def test_adam_several_steps_match_oracle(suco):
    # seven consecutive mini-batch steps over two epochs (a permuted order with
    # batches of 32, then row order with batches of 48, 48 and 32): moment decay
    # and bias correction past the first step, and the Adam state kept between
    # epochs, against the FP64 oracle taking the same batches with one state
    rng = np.random.default_rng(4)
    n_in, m = 9, 128
    net = suco.MLP(n_in, seed=6)
    F = rng.normal(size=(m, n_in)).astype(np.float32)
    t = rng.normal(size=m).astype(np.float32)
    perm = rng.permutation(m).astype(np.int32)
    ref = MLP64(split(net.params().astype(np.float64), n_in))
    state = {}
    batches = [perm[i:i + 32] for i in range(0, m, 32)] + [np.arange(i, min(m, i + 48)) for i in range(0, m, 48)]
    gmin = {k: np.full_like(v, np.inf) for k, v in ref.p.items()}
    gmax = {k: 0.0 for k in ref.p}
    for rows in batches:
        _, g = ref.loss_and_grad(F[rows], t[rows])
        for k in PARAM_NAMES:
            gmin[k] = np.minimum(gmin[k], np.abs(g[k]))
            gmax[k] = max(gmax[k], float(np.abs(g[k]).max()))
        ref.adam_step(g, state, lr=1e-3)
    Fd, td = torch.from_numpy(F).cuda(), torch.from_numpy(t).cuda()
    net.train_epoch(Fd, td, batch=32, lr=1e-3, order=torch.from_numpy(perm).cuda())
    net.train_epoch(Fd, td, batch=48, lr=1e-3)
    after = split(net.params().astype(np.float64), n_in)
    for k in PARAM_NAMES:
        big = gmin[k] > 1e-4 * gmax[k]
        assert big.mean() > 0.5, k
        assert np.allclose(after[k][big], ref.p[k][big], atol=2e-6, rtol=1e-5), k


def test_training_reduces_loss_on_a_learnable_target(suco):
    rng = np.random.default_rng(2)
    n_in, m = 17, 8192
    F = rng.normal(size=(m, n_in)).astype(np.float32)
    w = rng.normal(size=n_in)
    t = (np.tanh(F @ w / 4.0) - 4.0).astype(np.float32)    # log-alpha-like targets
    net = suco.MLP(n_in, seed=7)
    net.set_norm(F.mean(axis=0), F.std(axis=0))
    Fd, td = torch.from_numpy(F).cuda(), torch.from_numpy(t).cuda()
    l0 = net.train_epoch(Fd, td, batch=512, lr=1e-3)
    for _ in range(10):
        l1 = net.train_epoch(Fd, td, batch=512, lr=1e-3)
    assert l1 < 0.1 * l0


def test_bf16_inference_matches_oracle_model(suco):
    rng = np.random.default_rng(3)
    n_in, m = 17, 500
    net = suco.MLP(n_in, seed=11)
    mu = rng.normal(size=n_in).astype(np.float32)
    sd = (0.5 + rng.random(n_in)).astype(np.float32)
    net.set_norm(mu, sd)
    F = (rng.normal(size=(m, n_in)) * sd + mu).astype(np.float32)
    y, a = net.predict(torch.from_numpy(F).cuda(), scale=0.5, alpha_min=1e-3, alpha_max=0.2)
    torch.cuda.synchronize()
    ref = MLP64(split(net.params().astype(np.float64), n_in), mu=mu, sigma=sd)
    ry = ref.forward_bf16(F)
    assert np.abs(y.cpu().numpy() - ry).max() <= 5e-3
    ra = np.clip(0.5 * np.exp(y.cpu().numpy().astype(np.float64)), 1e-3, 0.2)
    assert np.allclose(a.cpu().numpy(), ra, rtol=1e-5)


def test_features_match_oracle(suco):
    W = synth.Workload(1)
    X, Q = W.data(), W.queries(50)
    _, c32, asg, _ = oracle.build_index(X, 8, 16, iters=6)
    oix = oracle.Index(X, 8, 16, c32, asg)
    ix = suco.Index.from_index(torch.from_numpy(X).cuda(), 8, 16, c32, asg)
    F = suco.query_features(ix, torch.from_numpy(Q).cuda()).cpu().numpy()
    for q in range(50):
        e = [np.sqrt(oix.centroid_dists(Q[q], g).min()) for g in range(16)]
        e.append(np.sqrt((Q[q].astype(np.float64) ** 2).sum()))
        assert np.allclose(F[q], e, rtol=1e-5, atol=1e-5)
    # the half distances are the activation step's own values, bit for bit
    o = ix.query_debug(torch.from_numpy(Q).cuda(), 10, 0.05, 0.005, scores=False, cand=False, cells=False)
    torch.cuda.synchronize()
    assert np.array_equal(F[:, :16], o["feat"].cpu().numpy())
    ix.free()


@pytest.mark.parametrize("d,ns,sk,nq", [(128, 8, 16, 300), (96, 8, 20, 33), (256, 4, 12, 50), (28, 3, 9, 16),
                                        (480, 15, 34, 40)])
def test_fused_alphas_equal_features_then_predict(suco, d, ns, sk, nq):
    """The query path's fused kernel (sixteen rows at a time when the widest
    half has at most 16 dimensions, else row by row) gives exactly the alphas
    of suco_query_features followed by suco_mlp_predict."""
    rng = np.random.default_rng(d + nq)
    X = rng.integers(0, 256, size=(3000, d)).astype(np.float32)
    Q = rng.integers(0, 256, size=(nq, d)).astype(np.float32)
    _, c32, asg, _ = oracle.build_index(X, ns, sk, iters=3)
    ix = suco.Index.from_index(torch.from_numpy(X).cuda(), ns, sk, c32, asg)
    Qd = torch.from_numpy(Q).cuda()
    net = suco.MLP(2 * ns + 1, seed=5)
    F = suco.query_features(ix, Qd)
    net.set_norm(F.mean(dim=0).cpu().numpy(), (F.std(dim=0) + 1.0).cpu().numpy())
    print(f"case: fused alphas d={d} ns={ns} sk={sk} nq={nq}", flush=True)
    _, a_ref = net.predict(F, 0.02, 0.001, 0.5)
    _, _, au = suco.query_learned(ix, net, Qd, 10, 0.01, 0.02, 0.001, 0.5)
    torch.cuda.synchronize()
    assert np.array_equal(au.cpu().numpy().view(np.uint32), a_ref.cpu().numpy().view(np.uint32))
    net.free()
    ix.free()


def test_learned_query_equals_plain_with_its_alphas(suco):
    """suco_query_learned = features + inference + the per-query-alpha path, exactly;
    and the batcher with the model attached gives the same results; and the oracle
    agrees with the GPU on those alphas."""
    W = synth.Workload(1)
    X, Q = W.data(), W.queries(300)
    _, c32, asg, _ = oracle.build_index(X, 8, 16, iters=6)
    oix = oracle.Index(X, 8, 16, c32, asg)
    ix = suco.Index.from_index(torch.from_numpy(X).cuda(), 8, 16, c32, asg)
    Qd = torch.from_numpy(Q).cuda()
    net = suco.MLP(17, seed=13)
    F = suco.query_features(ix, Qd)
    net.set_norm(F.mean(dim=0).cpu().numpy(), F.std(dim=0).cpu().numpy())
    ids, d, au = suco.query_learned(ix, net, Qd, 10, 0.01, 0.05, 0.005, 0.3)
    p_ids, p_d = ix.query_alpha(Qd, 10, au, 0.01)
    torch.cuda.synchronize()
    assert np.array_equal(ids.cpu().numpy(), p_ids.cpu().numpy())
    assert np.array_equal(d.cpu().numpy(), p_d.cpu().numpy())
    b = suco.Batcher(ix, 512, 10, 0.01)
    b.set_model(net, 0.05, 0.005, 0.3)
    b_ids, b_d = b.query(Qd)
    torch.cuda.synchronize()
    assert np.array_equal(b_ids.cpu().numpy(), ids.cpu().numpy())
    assert np.array_equal(b_d.cpu().numpy(), d.cpu().numpy())
    # uneven batches handed over together: each query's alpha is still its own
    outs = b.query_multi([Qd[:100], Qd[100:101], Qd[101:]])
    torch.cuda.synchronize()
    assert np.array_equal(torch.cat([o[0] for o in outs]).cpu().numpy(), ids.cpu().numpy())
    assert np.array_equal(torch.cat([o[1] for o in outs]).cpu().numpy(), d.cpu().numpy())
    b.free()
    aq = au.cpu().numpy()
    g = {kk: v.cpu().numpy() if v.dtype != torch.uint16 else v.view(torch.int16).cpu().numpy().view(np.uint16)
         for kk, v in ix.query_debug(Qd[:40], 10, 0.0, 0.01, alpha_q=au[:40]).items() if v is not None}
    check_query(oix, X, Q[:40], 10, aq[:40].astype(np.float64), 0.01, g)
    ix.free()


def test_trained_budget_gain_sift_like(suco):
    """SIFT-like 1M x 128: a network trained on plain-method labels reaches
    recall@10 >= 0.95 on held-out queries with a smaller mean alpha than the
    fixed alpha that reaches the same recall."""
    from paper_2411_14754_amd import learned
    W = synth.Workload(2)
    X = torch.from_numpy(W.data()).cuda()
    print("case: learned gain sift_like: build", flush=True)
    ix = suco.Index.build(X, 8, 50, iters=8)
    import bench
    Qt = torch.from_numpy(W.train_queries(24_000)).cuda()
    Qe = torch.from_numpy(W.queries(6_000)).cuda()
    gt_t = bench.exact_topk(X, Qt, 10)
    gt_e = bench.exact_topk(X, Qe, 10)
    grid = learned.alpha_grid(0.0005, 0.05)
    print("case: learned gain: labels and training", flush=True)
    net, info = learned.train_budget_model(ix, Qt[:20_000], gt_t[:20_000], 10, 0.005, grid, epochs=25)
    assert info["loss"][-1] < info["loss"][0]
    scale = learned.calibrate_scale(ix, net, Qt[20_000:], gt_t[20_000:], 10, 0.005, 0.95, 0.0005, 0.05)
    ids, _, au = suco.query_learned(ix, net, Qe, 10, 0.005, scale, 0.0005, 0.05)
    r_learned = float(learned.per_query_recall(ids, gt_e).mean())
    mean_alpha = float(au.double().mean())
    # the fixed alpha that reaches the same recall on these queries
    fixed = None
    for a in learned.alpha_grid(0.0005, 0.05, 1.1):
        pi, _ = ix.query(Qe, 10, a, 0.005)
        if float(learned.per_query_recall(pi, gt_e).mean()) >= r_learned:
            fixed = a
            break
    print(f"learned: recall {r_learned:.4f} mean alpha {mean_alpha:.5f}; fixed alpha for that recall {fixed}",
          flush=True)
    assert r_learned >= 0.94
    assert fixed is not None and mean_alpha < fixed
    ix.free()


def test_trained_budget_lifted_reduced(suco):
    """The lifted generator (d = 256, N_s = 16, sqrtK = 64) at n = 1,000,000:
    a network trained on plain-method labels and calibrated on held-out
    queries reaches recall@10 >= 0.94 on other queries with per-query alphas
    that vary, and its query equals the per-query-alpha path on those alphas.
    At this size it does not beat a fixed alpha (mean alpha ~0.00105 against
    ~0.00087 for the same recall, printed), so no gain is asserted."""
    from paper_2411_14754_amd import learned
    W = synth.Workload(5)
    X = torch.from_numpy(W.data(1_000_000)).cuda()
    print("case: learned lifted n=1e6: build", flush=True)
    ix = suco.Index.build(X, 16, 64, iters=6)
    import bench
    Qt = torch.from_numpy(W.train_queries(24_000)).cuda()
    Qe = torch.from_numpy(W.queries(4_000)).cuda()
    gt_t = bench.exact_topk_float(X, Qt, 10)
    gt_e = bench.exact_topk_float(X, Qe, 10)
    grid = learned.alpha_grid(0.00005, 0.02, 1.4)
    print("case: learned lifted: labels and training", flush=True)
    net, info = learned.train_budget_model(ix, Qt[:20_000], gt_t[:20_000], 10, 0.003, grid, epochs=25)
    assert info["loss"][-1] < info["loss"][0]
    scale = learned.calibrate_scale(ix, net, Qt[20_000:], gt_t[20_000:], 10, 0.003, 0.95, grid[0], grid[-1])
    ids, dists, au = suco.query_learned(ix, net, Qe, 10, 0.003, scale, grid[0], grid[-1])
    r_learned = float(learned.per_query_recall(ids, gt_e).mean())
    mean_alpha = float(au.double().mean())
    p_ids, p_d = ix.query_alpha(Qe, 10, au, 0.003)
    torch.cuda.synchronize()
    assert torch.equal(ids, p_ids) and torch.equal(dists, p_d)
    fixed = None
    for a in learned.alpha_grid(grid[0], grid[-1], 1.1):
        pi, _ = ix.query(Qe, 10, a, 0.003)
        if float(learned.per_query_recall(pi, gt_e).mean()) >= r_learned:
            fixed = a
            break
    print(f"learned (lifted n=1e6): recall {r_learned:.4f} mean alpha {mean_alpha:.6f}; fixed alpha for that "
          f"recall {fixed}", flush=True)
    assert r_learned >= 0.94
    assert float(au.double().std()) > 0.1 * mean_alpha
    ix.free()
