"""Pins of the FP64 warm-start MLP oracle: finite differences of the loss,
closed forms, the Adam update against its definition on a scalar, and the
column features against direct per-column formulas. CPU only."""
import numpy as np
import pytest

from oracle import goat_oracle as O
from oracle import mlp_oracle as M


def _params(seed=0, scale=1.0):
    p = M.init_params(seed)
    rng = np.random.default_rng(seed + 1)
    for k in ("b1", "b2", "b3"):
        p[k] = 0.1 * rng.normal(size=p[k].shape)
    return {k: v * scale for k, v in p.items()}


def test_forward_zero_weights_is_bias():
    p = _params()
    for k in ("W1", "W2", "W3"):
        p[k] = np.zeros_like(p[k])
    F = np.random.default_rng(3).normal(size=(7, 4))
    y, _ = M.forward(p, F)
    assert np.allclose(y, p["b3"][0])


def test_forward_linear_regime():
    """With all pre-activations positive the network is affine: y is
    W3 W2 W1 F + (W3 W2 b1 + W3 b2 + b3)."""
    rng = np.random.default_rng(4)
    p = dict(W1=np.abs(rng.normal(size=(128, 4))), b1=np.abs(rng.normal(size=128)) + 1,
             W2=np.abs(rng.normal(size=(128, 128))), b2=np.abs(rng.normal(size=128)) + 1,
             W3=rng.normal(size=(1, 128)), b3=rng.normal(size=1))
    F = np.abs(rng.normal(size=(5, 4)))
    y, _ = M.forward(p, F)
    lin = (F @ (p["W3"] @ p["W2"] @ p["W1"]).T)[:, 0] + (p["W3"] @ (p["W2"] @ p["b1"] + p["b2"]))[0] + p["b3"][0]
    assert np.allclose(y, lin, rtol=1e-12)


def test_backward_matches_finite_differences():
    p = _params(7)
    rng = np.random.default_rng(8)
    F = rng.normal(size=(33, 4))
    t = rng.normal(size=33)
    L, g = M.loss_and_grads(p, F, t)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        idx = rng.choice(flat.size, size=min(6, flat.size), replace=False)
        for j in idx:
            old = flat[j]
            flat[j] = old + h
            Lp, _ = M.loss_and_grads(p, F, t)
            flat[j] = old - h
            Lm, _ = M.loss_and_grads(p, F, t)
            flat[j] = old
            fd = (Lp - Lm) / (2 * h)
            assert g[k].reshape(-1)[j] == pytest.approx(fd, rel=1e-5, abs=1e-8), (k, j)


def test_adam_scalar_definition():
    """First Adam step moves every parameter by -lr * sign(g) (bias
    correction makes mh/sqrt(vh) = g/|g|)."""
    p = dict(w=np.array([1.0, -2.0, 3.0]))
    g = dict(w=np.array([0.5, -4.0, 1e-3]))
    m = dict(w=np.zeros(3)); v = dict(w=np.zeros(3))
    M.adam_step(p, g, m, v, step=1, lr=0.1)
    assert np.allclose(p["w"], [0.9, -1.9, 2.9], atol=1e-6)


def test_training_reduces_loss():
    rng = np.random.default_rng(11)
    F = rng.normal(size=(256, 4))
    t = np.sin(F[:, 0]) + 0.5 * F[:, 3]
    p = M.init_params(1)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(x) for k, x in p.items()}
    L0, _ = M.loss_and_grads(p, F, t)
    for step in range(1, 201):
        _, g = M.loss_and_grads(p, F, t)
        M.adam_step(p, g, m, v, step, 3e-3)
    L1, _ = M.loss_and_grads(p, F, t)
    assert L1 < 0.2 * L0


def test_column_features_direct():
    rng = np.random.default_rng(12)
    n = 17
    G = rng.normal(size=(n, n)) * 5
    eps = 0.7
    F = M.column_features(G, eps)
    X = G / eps
    j = 5
    col = X[:, j]
    raw = np.array([col.mean(), col.max(), col.std(), np.log(np.mean(np.exp(col)))])
    allraw = np.array([[X[:, c].mean(), X[:, c].max(), X[:, c].std(), np.log(np.mean(np.exp(X[:, c])))]
                       for c in range(n)])
    assert np.allclose(F[j], raw - allraw.mean(axis=0), rtol=1e-12, atol=1e-12)
    assert np.allclose(F.mean(axis=0), 0.0, atol=1e-12)


def test_lse_feature_is_first_column_update():
    """With f = 0 the first column update of the log-domain Sinkhorn is
    g_j / eps = -LSE_i(G_ij / eps): the centred LSE feature equals the
    centred negative of that potential - the trivial warm start the MLP
    improves on."""
    rng = np.random.default_rng(13)
    n = 30
    G = rng.random((n, n))
    eps = 0.1
    F = M.column_features(G, eps)
    g1 = -eps * np.log(np.sum(np.exp(G / eps), axis=0))
    assert np.allclose(F[:, 3], -M.centred_target(g1, eps), atol=1e-10)
