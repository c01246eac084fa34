"""Seeded synthetic inputs shared by the HIP path, the oracle and the benchmark.

This module only draws random numbers and lays them out as graph pairs; it
holds none of the matching method's arithmetic (no gradient, no Sinkhorn
scaling, no assignment). Both sides of every parity test receive the same
bytes from here.

Graph model: the rho-correlated stochastic block model of the paper's
"Correlated Network Simulation Setup" section. For every unordered node pair
i < j with block edge probability p, draw A_ij ~ Bernoulli(p); the aligned copy
B'_ij is Bernoulli(p + rho (1 - p)) where A_ij = 1 and Bernoulli(p (1 - rho))
where A_ij = 0, so B' has the same edge density p and edge correlation rho with
A. Graphs are simple and undirected (symmetric, zero diagonal). The
Erdos-Renyi model is the one-block case. B is then B' with its nodes shuffled
by a seeded uniform permutation pi: B = B'[pi][:, pi], so A-node i corresponds
to B-node argsort(pi)[i].

Weighted variant (stand-in for the weighted 10,000-node email subgraphs of the
"Organization Email Network" section, a private dataset): A has block-model
support with symmetric weights exp(z), z ~ N(0, 1); B' = A + E with symmetric
E ~ N(0, sigma^2) on A's support only, so B' shares A's edges.

Arrays are returned as float32 (the GPU path's storage type). The oracle
promotes them exactly to float64.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SEED_BASE = 20211105


@dataclass
class GraphPair:
    A: np.ndarray          # float32 n x n, symmetric
    B: np.ndarray          # float32 n x n, symmetric, nodes shuffled
    truth: np.ndarray      # int64 [n]: A-node i corresponds to B-node truth[i]
    meta: dict


def _block_prob_matrix(block_sizes, block_probs) -> np.ndarray:
    sizes = np.asarray(block_sizes, dtype=np.int64)
    bp = np.asarray(block_probs, dtype=np.float64)
    labels = np.repeat(np.arange(len(sizes)), sizes)
    return labels, bp


def _upper_mask(n: int) -> np.ndarray:
    return np.triu(np.ones((n, n), dtype=bool), k=1)


def _correlated_support(rng, n, labels, bp, rho):
    """Upper-triangular boolean supports (a, b') of a rho-correlated pair."""
    iu, ju = np.triu_indices(n, k=1)
    p = bp[labels[iu], labels[ju]]
    ua = rng.random(iu.shape[0])
    a = ua < p
    ub = rng.random(iu.shape[0])
    pb = np.where(a, p + rho * (1.0 - p), p * (1.0 - rho))
    b = ub < pb
    return iu, ju, a, b


def _symmetric_from_upper(n, iu, ju, vals, dtype=np.float32):
    M = np.zeros((n, n), dtype=dtype)
    M[iu, ju] = vals
    M[ju, iu] = vals
    return M


def rho_sbm_pair(block_sizes, block_probs, rho: float, seed: int,
                 perm_seed: int | None = None) -> GraphPair:
    """0/1 rho-correlated SBM pair, B shuffled by a seeded permutation."""
    labels, bp = _block_prob_matrix(block_sizes, block_probs)
    n = labels.shape[0]
    rng = np.random.default_rng(seed)
    iu, ju, a, b = _correlated_support(rng, n, labels, bp, rho)
    A = _symmetric_from_upper(n, iu, ju, a.astype(np.float32))
    Bp = _symmetric_from_upper(n, iu, ju, b.astype(np.float32))
    prng = np.random.default_rng(seed + 100 if perm_seed is None else perm_seed)
    pi = prng.permutation(n)
    B = np.ascontiguousarray(Bp[np.ix_(pi, pi)])
    truth = np.argsort(pi)
    return GraphPair(A, B, truth, dict(kind="rho-sbm", n=n, rho=rho, seed=seed,
                                       block_sizes=list(map(int, block_sizes))))


def rho_er_pair(n: int, p: float, rho: float, seed: int,
                perm_seed: int | None = None) -> GraphPair:
    """0/1 rho-correlated Erdos-Renyi pair (the one-block SBM)."""
    g = rho_sbm_pair([n], [[p]], rho, seed, perm_seed)
    g.meta.update(kind="rho-er", p=p)
    return g


def weighted_sbm_pair(block_sizes, block_probs, sigma: float, seed: int,
                      perm_seed: int | None = None) -> GraphPair:
    """Weighted SBM pair: lognormal(0,1) weights on A; B' = A + N(0, sigma^2)
    on A's edges; B = B' shuffled."""
    labels, bp = _block_prob_matrix(block_sizes, block_probs)
    n = labels.shape[0]
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, k=1)
    p = bp[labels[iu], labels[ju]]
    edge = rng.random(iu.shape[0]) < p
    iu, ju = iu[edge], ju[edge]
    w = np.exp(rng.standard_normal(iu.shape[0]))
    e = sigma * rng.standard_normal(iu.shape[0])
    A = _symmetric_from_upper(n, iu, ju, w.astype(np.float32))
    Bp = _symmetric_from_upper(n, iu, ju, (w + e).astype(np.float32))
    prng = np.random.default_rng(seed + 100 if perm_seed is None else perm_seed)
    pi = prng.permutation(n)
    B = np.ascontiguousarray(Bp[np.ix_(pi, pi)])
    truth = np.argsort(pi)
    return GraphPair(A, B, truth, dict(kind="weighted-sbm", n=n, sigma=sigma, seed=seed,
                                       block_sizes=list(map(int, block_sizes))))


def uniform_matrix(n: int, seed: int) -> np.ndarray:
    """U(0,1) n x n draw (float32) for random doubly stochastic inits."""
    rng = np.random.default_rng(seed)
    return rng.random((n, n)).astype(np.float32)


def cost_matrix(n: int, seed: int, lo: float = 100.0, hi: float = 150.0) -> np.ndarray:
    """n x n costs drawn from Uniform(lo, hi) (float32): the cost matrices of
    the LOT-versus-LAP comparison (Uniform(100, 150))."""
    rng = np.random.default_rng(SEED_BASE + 700 + seed)
    return (lo + (hi - lo) * rng.random((n, n))).astype(np.float32)


def random_matrix(m: int, n: int, seed: int, lo: float = -1.0, hi: float = 1.0,
                  dtype=np.float32) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (lo + (hi - lo) * rng.random((m, n))).astype(dtype)


def random_doubly_stochastic_draws(n: int, seed: int, terms: int = 4):
    """Weights and permutations for a random convex combination of
    permutation matrices (a point of the Birkhoff polytope): returns
    (weights[terms] summing to 1, perms[terms, n])."""
    rng = np.random.default_rng(seed)
    w = rng.random(terms) + 0.1
    w = w / w.sum()
    perms = np.stack([rng.permutation(n) for _ in range(terms)])
    return w, perms


# ---- named workloads -------------------------------------------------------

def workload_er_small(config_seed_offset: int = 1) -> GraphPair:
    """n=64 correlated ER pair, p=0.1, rho=0.9."""
    return rho_er_pair(64, 0.1, 0.9, SEED_BASE + config_seed_offset)


def workload_er_2000() -> GraphPair:
    """n=2000 correlated ER pair, p=0.01, rho=0.8."""
    return rho_er_pair(2000, 0.01, 0.8, SEED_BASE + 2)


def workload_weighted_sbm(n: int = 10000) -> GraphPair:
    """4-block weighted SBM, in-block 0.02, out-of-block 0.005, equal blocks."""
    k = 4
    sizes = [n // k + (1 if r < n % k else 0) for r in range(k)]
    bp = np.full((k, k), 0.005)
    np.fill_diagonal(bp, 0.02)
    return weighted_sbm_pair(sizes, bp, 0.1, SEED_BASE + 3)


def workload_er_5000() -> GraphPair:
    """n=5000 correlated ER pair, p=0.02, rho=0.7."""
    return rho_er_pair(5000, 0.02, 0.7, SEED_BASE + 5)


def workload_batch(npairs: int = 512, restarts: int = 8, n_lo: int = 50, n_hi: int = 400,
                   seed_offset: int = 4):
    """Random-start batch: npairs correlated ER pairs with n ~ U{n_lo..n_hi},
    p ~ U(0.05, 0.3), rho ~ U(0.6, 1.0), each with `restarts` U(0,1) n x n
    draws for the random starts, stacked as a (restarts*n, n) float32 array.
    Returns a list of (GraphPair, U)."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    out = []
    for _ in range(npairs):
        n = int(rng.integers(n_lo, n_hi + 1))
        p = float(rng.uniform(0.05, 0.3))
        rho = float(rng.uniform(0.6, 1.0))
        s = int(rng.integers(0, 2 ** 31 - 1))
        g = rho_er_pair(n, p, rho, s)
        U = np.random.default_rng(s + 7).random((restarts * n, n)).astype(np.float32)
        out.append((g, U))
    return out


def mlp_init_params(seed: int, hidden: int = 128, nfeat: int = 4) -> np.ndarray:
    """Packed float32 initial weights of the warm-start network
    (W1[h][f], b1, W2[h][h], b2, W3[h], b3): normal draws with He scaling,
    zero biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0.0, np.sqrt(2.0 / nfeat), size=(hidden, nfeat))
    W2 = rng.normal(0.0, np.sqrt(2.0 / hidden), size=(hidden, hidden))
    W3 = rng.normal(0.0, np.sqrt(1.0 / hidden), size=(hidden,))
    z = np.zeros
    return np.concatenate([W1.ravel(), z(hidden), W2.ravel(), z(hidden), W3, z(1)]).astype(np.float32)
