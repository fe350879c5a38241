"""Training and calibration of the learned activation budget.

Labels come from the plain method itself: for each training query, the
smallest collision ratio on a geometric grid whose top-k equals the exact
top-k (per-query recall@k = 1), or the grid's largest value if none does.  The
network regresses log alpha on the query features (mean squared error), and a
global scale on the predicted alpha is calibrated on held-out queries so that
their mean recall@k reaches the target.  Every query and every training step
runs in the library's kernels; this module only drives them.
"""
from __future__ import annotations

import math

import numpy as np

from . import MLP, Index, query_features, query_learned


def alpha_grid(lo: float, hi: float, ratio: float = 1.25) -> list[float]:
    n = int(math.floor(math.log(hi / lo) / math.log(ratio) + 1e-9)) + 1
    return [lo * ratio ** j for j in range(n)]


def per_query_recall(ids, gt):
    """|R intersect R*| / k for every query (torch tensors [nq, k])."""
    k = gt.shape[1]
    return (ids[:, :, None] == gt[:, None, :]).any(dim=2).sum(dim=1).float() / k


def label_alphas(index: Index, Q, gt, k: int, beta: float, grid: list[float], chunk: int = 16384):
    """Per query, the smallest grid alpha whose recall@k equals the recall at
    the grid's largest alpha: where the query's recall stops improving.  (A
    query that the candidate budget beta*n never lets reach recall 1 is not
    pushed to the largest alpha.)"""
    import torch
    nq = Q.shape[0]
    grid = sorted(grid)
    best = torch.empty(nq, dtype=torch.float32, device="cuda")
    for s in range(0, nq, chunk):
        e = min(nq, s + chunk)
        ids, _ = index.query(Q[s:e], k, grid[-1], beta)
        best[s:e] = per_query_recall(ids, gt[s:e])
    label = torch.full((nq,), float(grid[-1]), dtype=torch.float32, device="cuda")
    done = torch.zeros(nq, dtype=torch.bool, device="cuda")
    for a in grid:
        for s in range(0, nq, chunk):
            e = min(nq, s + chunk)
            todo = ~done[s:e]
            if not bool(todo.any()):
                continue
            ids, _ = index.query(Q[s:e], k, a, beta)
            hit = (per_query_recall(ids, gt[s:e]) >= best[s:e]) & todo
            label[s:e][hit] = a
            done[s:e] |= hit
    return label


def fit(mlp: MLP, F, y, epochs: int = 30, batch: int = 1024, lr: float = 1e-3, seed: int = 0):
    """Standardise the features, then mini-batch Adam on (F, y); returns the loss per epoch."""
    import torch
    Fh = F.double()
    mu = Fh.mean(dim=0).float().cpu().numpy()
    sd = Fh.std(dim=0).clamp_min(1e-6).float().cpu().numpy()
    mlp.set_norm(mu, sd)
    rng = np.random.Generator(np.random.PCG64(seed))
    m = F.shape[0]
    hist = []
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(m).astype(np.int32)).cuda()
        hist.append(mlp.train_epoch(F, y, batch, lr, order=order, want_loss=(ep == epochs - 1 or ep % 5 == 0)))
    return hist


def calibrate_scale(index: Index, mlp: MLP, Q, gt, k: int, beta: float, target: float, alpha_min: float,
                    alpha_max: float, lo: float = 0.05, hi: float = 50.0, steps: int = 14):
    """Smallest scale (bisection in log space) whose mean recall@k on (Q, gt) reaches target."""
    def rec(s):
        ids, _, _ = query_learned(index, mlp, Q, k, beta, s, alpha_min, alpha_max)
        return float(per_query_recall(ids, gt).mean())
    if rec(hi) < target:
        return hi
    a, b = math.log(lo), math.log(hi)
    for _ in range(steps):
        mid = 0.5 * (a + b)
        if rec(math.exp(mid)) >= target:
            b = mid
        else:
            a = mid
    return math.exp(b)


def train_budget_model(index: Index, Q_train, gt_train, k: int, beta: float, grid: list[float],
                       epochs: int = 30, batch: int = 1024, lr: float = 1e-3, seed: int = 0):
    """Labels from plain sweeps, features from the index, and a trained MLP."""
    import torch
    labels = label_alphas(index, Q_train, gt_train, k, beta, grid)
    F = query_features(index, Q_train)
    y = torch.log(labels)
    mlp = MLP(2 * index.ns + 1, seed=seed + 1)
    hist = fit(mlp, F, y, epochs=epochs, batch=batch, lr=lr, seed=seed)
    return mlp, {"labels": labels, "loss": hist}
