"""FP64 oracle of the learned activation-budget network -- TEST INFRASTRUCTURE ONLY.

The paper fixes one collision ratio alpha for all queries and names combining
the method with learned models as future work (Sec. 6).  The learned form
predicts a per-query alpha with a small MLP:

    x      = (features - mu) / sigma                       (fixed standardisation)
    h1     = GELU(W1 x + b1)          W1: [H, n_in]
    h2     = GELU(W2 h1 + b2)         W2: [H, H]
    y      = W3 h2 + b3               W3: [1, H]   (y predicts log alpha)
    loss   = mean_i (y_i - t_i)^2

GELU(x) = x * Phi(x) with the exact normal CDF (Hendrycks & Gimpel 2016).
Adam follows Kingma & Ba (2015), Algorithm 1, with bias correction.
Everything here is FP64 NumPy; the gradients are the analytic chain rule.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT1_2 = 1.0 / math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(x):
    return x * 0.5 * (1.0 + erf(x * SQRT1_2))


def gelu_grad(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + erf(x * SQRT1_2)) + x * INV_SQRT_2PI * np.exp(-0.5 * x * x)


PARAM_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


class MLP64:
    def __init__(self, params: dict, mu=None, sigma=None):
        self.p = {k: np.array(params[k], np.float64) for k in PARAM_NAMES}
        n_in = self.p["W1"].shape[1]
        self.mu = np.zeros(n_in) if mu is None else np.asarray(mu, np.float64)
        self.sigma = np.ones(n_in) if sigma is None else np.asarray(sigma, np.float64)

    def standardise(self, F):
        return (np.asarray(F, np.float64) - self.mu) / self.sigma

    def forward(self, F, keep=False):
        p = self.p
        x = self.standardise(F)
        z1 = x @ p["W1"].T + p["b1"]
        h1 = gelu(z1)
        z2 = h1 @ p["W2"].T + p["b2"]
        h2 = gelu(z2)
        y = (h2 @ p["W3"].T + p["b3"])[:, 0]
        if keep:
            return y, (x, z1, h1, z2, h2)
        return y

    def forward_bf16(self, F):
        """BF16 inference model: parameters and each layer's input rounded to
        BF16 (the standardised features in FP32 first), products and sums in
        FP64, GELU in FP64 and its output rounded to BF16 through FP32."""
        p = {k: bf16_round(np.asarray(v, np.float32)).astype(np.float64) for k, v in self.p.items()}
        x32 = (np.asarray(F, np.float32) - self.mu.astype(np.float32)) / self.sigma.astype(np.float32)
        x = bf16_round(x32).astype(np.float64)
        h1 = bf16_round(gelu(x @ p["W1"].T + p["b1"]).astype(np.float32)).astype(np.float64)
        h2 = bf16_round(gelu(h1 @ p["W2"].T + p["b2"]).astype(np.float32)).astype(np.float64)
        return (h2 @ p["W3"].T + p["b3"])[:, 0]

    def loss_and_grad(self, F, t):
        """MSE loss and its analytic gradient with respect to every parameter."""
        p = self.p
        y, (x, z1, h1, z2, h2) = self.forward(F, keep=True)
        m = y.shape[0]
        r = y - np.asarray(t, np.float64)
        loss = float(np.mean(r * r))
        dy = (2.0 / m) * r[:, None]                  # [m,1]
        g = {}
        g["W3"] = dy.T @ h2
        g["b3"] = dy.sum(axis=0)
        dh2 = dy @ p["W3"]
        dz2 = dh2 * gelu_grad(z2)
        g["W2"] = dz2.T @ h1
        g["b2"] = dz2.sum(axis=0)
        dh1 = dz2 @ p["W2"]
        dz1 = dh1 * gelu_grad(z1)
        g["W1"] = dz1.T @ x
        g["b1"] = dz1.sum(axis=0)
        return loss, g

    def adam_step(self, g, state, lr, b1=0.9, b2=0.999, eps=1e-8):
        state["t"] = state.get("t", 0) + 1
        tt = state["t"]
        for k in PARAM_NAMES:
            m = state.setdefault("m_" + k, np.zeros_like(self.p[k]))
            v = state.setdefault("v_" + k, np.zeros_like(self.p[k]))
            m[...] = b1 * m + (1.0 - b1) * g[k]
            v[...] = b2 * v + (1.0 - b2) * g[k] * g[k]
            mh = m / (1.0 - b1 ** tt)
            vh = v / (1.0 - b2 ** tt)
            self.p[k] = self.p[k] - lr * mh / (np.sqrt(vh) + eps)


def init_params(n_in: int, hidden: int, seed: int) -> dict:
    """He-style uniform initialisation from a seeded NumPy generator (FP32 values)."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def u(shape, fan_in):
        b = math.sqrt(3.0 / fan_in)
        return rng.uniform(-b, b, size=shape).astype(np.float32)

    return dict(W1=u((hidden, n_in), n_in), b1=np.zeros(hidden, np.float32),
                W2=u((hidden, hidden), hidden), b2=np.zeros(hidden, np.float32),
                W3=u((1, hidden), hidden), b3=np.zeros(1, np.float32))


def bf16_round(x) -> np.ndarray:
    """Round FP32 values to the nearest BF16 (ties to even), returned as FP32.

    BF16 keeps the top 16 bits of the IEEE-754 binary32 pattern; rounding to
    nearest-even adds 0x7FFF plus the lowest kept bit before truncating.
    """
    a = np.ascontiguousarray(x, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((u >> 16) & 1)
    r = ((u + bias) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    nan = np.isnan(a)
    if nan.any():
        out = out.copy()
        out[nan] = np.nan
    return out
