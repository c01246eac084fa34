"""FP64 CPU oracle for the learned Sinkhorn warm start.

TEST INFRASTRUCTURE ONLY (see goat_oracle.py): never imported by the
product path; shares no code with the HIP kernels.

The warm start maps per-column statistics of the scaled gradient
X = G / eps to the column dual potential g_j / eps of the converged Sinkhorn
solve (Alg. 2 with the cost negated). The paper does not describe it; the
readings are:
  * features of column j, from x_ij = G_ij / eps over rows i:
      mean_i x_ij,  max_i x_ij,  std_i x_ij (population),
      LSE_i x_ij - log n   (log-mean-exp),
    each then centred by subtracting its mean over j (the duals are defined
    up to a constant shift between f and g, so only differences matter);
  * target: g_j / eps of the converged solve, centred over j;
  * network: 4 -> 128 -> 128 -> 1, ReLU after the two hidden layers,
    float weights, loss = mean squared error over a batch;
  * optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias correction.
"""
from __future__ import annotations

import numpy as np

H = 128
NFEAT = 4


def column_features(G, eps):
    """Centred per-column features of X = G / eps (see module docstring)."""
    X = np.asarray(G, np.float64) / eps
    n = X.shape[0]
    mean = X.mean(axis=0)
    mx = X.max(axis=0)
    std = np.sqrt(np.mean((X - mean[None, :]) ** 2, axis=0))
    lse = mx + np.log(np.sum(np.exp(X - mx[None, :]), axis=0)) - np.log(n)
    F = np.stack([mean, mx, std, lse], axis=1)
    return F - F.mean(axis=0, keepdims=True)


def centred_target(g, eps):
    t = np.asarray(g, np.float64) / eps
    return t - t.mean()


def init_params(seed: int):
    """He-style initial weights (the GPU side receives these same values)."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0.0, np.sqrt(2.0 / NFEAT), size=(H, NFEAT))
    b1 = np.zeros(H)
    W2 = rng.normal(0.0, np.sqrt(2.0 / H), size=(H, H))
    b2 = np.zeros(H)
    W3 = rng.normal(0.0, np.sqrt(1.0 / H), size=(1, H))
    b3 = np.zeros(1)
    return dict(W1=W1, b1=b1, W2=W2, b2=b2, W3=W3, b3=b3)


def forward(p, F):
    """Returns (prediction [N], cache). F: [N, 4]."""
    F = np.asarray(F, np.float64)
    z1 = F @ p["W1"].T + p["b1"]
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ p["W2"].T + p["b2"]
    a2 = np.maximum(z2, 0.0)
    y = a2 @ p["W3"].T + p["b3"]
    return y[:, 0], (F, z1, a1, z2, a2)


def loss_and_grads(p, F, t):
    """MSE loss L = mean_k (y_k - t_k)^2 and its gradients by the chain rule."""
    y, (F, z1, a1, z2, a2) = forward(p, F)
    N = y.shape[0]
    r = y - np.asarray(t, np.float64)
    L = float(np.mean(r * r))
    dy = (2.0 / N) * r[:, None]                   # [N,1]
    g = {}
    g["W3"] = dy.T @ a2
    g["b3"] = dy.sum(axis=0)
    da2 = dy @ p["W3"]
    dz2 = da2 * (z2 > 0)
    g["W2"] = dz2.T @ a1
    g["b2"] = dz2.sum(axis=0)
    da1 = dz2 @ p["W2"]
    dz1 = da1 * (z1 > 0)
    g["W1"] = dz1.T @ F
    g["b1"] = dz1.sum(axis=0)
    return L, g


def adam_step(p, g, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of every parameter (in place); step counts from 1."""
    for k in p:
        m[k] = beta1 * m[k] + (1.0 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k]
        mh = m[k] / (1.0 - beta1 ** step)
        vh = v[k] / (1.0 - beta2 ** step)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def unpack(flat):
    """Parameter dict from the flat float32 vector the library stores
    (W1[128][4], b1[128], W2[128][128], b2[128], W3[128], b3[1], row-major),
    promoted exactly to float64."""
    x = np.asarray(flat, np.float64).ravel()
    sizes = [("W1", (H, NFEAT)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (1, H)), ("b3", (1,))]
    p, o = {}, 0
    for name, shape in sizes:
        k = int(np.prod(shape))
        p[name] = x[o:o + k].reshape(shape)
        o += k
    if o != x.size:
        raise ValueError(f"{x.size} parameters, expected {o}")
    return p


def warm_start(G, eps, p):
    """Column potentials g0 = eps * network(features of G / eps) that start a
    warm Sinkhorn solve (the network predicts the centred g / eps)."""
    y, _ = forward(p, column_features(G, eps))
    return eps * y


def network(flat):
    """warm_start as a function of (G, eps), for goat_oracle.goat(net=...)."""
    p = unpack(flat)
    return lambda G, eps: warm_start(G, eps, p)
