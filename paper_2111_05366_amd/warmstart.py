"""Training and use of the learned Sinkhorn warm start.

Training pairs come from the plain solver: on seeded correlated
Erdos-Renyi pairs, the gradient grad f(P) at each Frank-Wolfe iterate is
taken from the solver, solved to convergence by goat_sinkhorn (cold start),
and turned into (centred column features, centred g / eps) samples with
goat_mlp_features. The network is trained on the GPU by the library's own
backward and Adam kernels; this module only sequences the calls.
Parameters are stored with safetensors (flat float32 plus a JSON header).
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import goat, inputs

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PATH = os.path.join(HERE, "data", "warmstart_mlp.safetensors")


def _torch():
    import torch
    return torch


def _pair_edges(spec):
    """Worker: the seeded pair of `spec` = (n, p, rho, seed) as the upper
    triangles' nonzero positions of A and B (both symmetric 0/1, hollow), so
    that a worker process sends a few MB instead of two dense matrices."""
    n, p, rho, seed = spec
    g = inputs.rho_er_pair(n, p, rho, seed)
    out = [n, seed]
    for X in (g.A, g.B):
        iu, ju = np.nonzero(np.triu(X, 1))
        out.append((iu.astype(np.int32) * np.int64(n) + ju).astype(np.int64))
    return tuple(out)


def _dense_from_edges(n, flat, torch):
    X = torch.zeros(n * n, dtype=torch.float32, device="cuda")
    idx = torch.as_tensor(flat, device="cuda")
    X[idx] = 1.0
    X = X.view(n, n)
    return X + X.t()


def _pairs_stream(pairs, workers):
    """(n, seed, A, B) device tensors for each pair spec, drawn by `workers`
    spawned processes (0: in this process)."""
    torch = _torch()
    if workers <= 0:
        for (n, p, rho, seed) in pairs:
            g = inputs.rho_er_pair(n, p, rho, seed)
            yield n, seed, torch.as_tensor(g.A, device="cuda"), torch.as_tensor(g.B, device="cuda")
        return
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(workers) as pool:
        for (n, seed, ea, eb) in pool.imap(_pair_edges, pairs, chunksize=1):
            yield n, seed, _dense_from_edges(n, ea, torch), _dense_from_edges(n, eb, torch)


def generate(pairs, fw_iters: int = 6, sk_tol: float = 1e-6, sk_cap: int = 3000, eps_rel: float = 0.03,
             log=None, max_solves: int = 0, workers: int = 0):
    """Samples (F [N,4], target [N], solves) from a list of (n, p, rho, seed).
    Each FW iterate of the plain fp32 solver gives one Sinkhorn problem;
    iterates after a zero step (same G as before) and solves that did not
    reach sk_tol within sk_cap are skipped (their g is not the fixed point).
    Stops after max_solves kept solves (0: all pairs); pairs are drawn by
    `workers` processes."""
    torch = _torch()
    feats, targs, meta = [], [], []
    for (n, seed, A, B) in _pairs_stream(pairs, workers):
        run = goat.Run(A, B, prec="fp32", sk_max=1000, stop_on_stall=1, eps_rel=eps_rel)
        kept = []
        for k in range(fw_iters):
            G = run.gradient()
            out = goat.sinkhorn(G, eps_rel=eps_rel, max_iter=sk_cap, tol=sk_tol, want_Q=False)
            iters, err = int(out.iters.item()), float(out.err.item())
            if err <= sk_tol:
                eps = out.eps
                F = goat.mlp_features(G, eps)
                t = out.g / eps
                feats.append(F)
                targs.append(t - t.mean())
                meta.append(dict(n=n, seed=seed, fw=k, iters=iters, err=err))
                kept.append(iters)
            if run.steps(1) == 0 or run.history[-1]["t"] == 0.0:
                break   # a zero step leaves P, hence G, unchanged
        run.close()
        del A, B
        if log:
            log(f"warmstart data: n={n} seed={seed} kept solves (iters) {kept}; {len(meta)} solves so far")
        if max_solves and len(meta) >= max_solves:
            break
    return torch.cat(feats), torch.cat(targs), meta


def training_pairs(count: int = 48, seed: int = 0):
    """(n, p, rho, seed) of the learned-part training set: correlated ER
    pairs with n uniform in [500, 5000], p = 0.02, rho = 0.7."""
    rng = np.random.default_rng(inputs.SEED_BASE + 600 + seed)
    return [(int(rng.integers(500, 5001)), 0.02, 0.7, inputs.SEED_BASE + 1000 + i) for i in range(count)]


# Pair seeds of the training set start at SEED_BASE + 1000; held-out pairs
# must lie outside [SEED_BASE + 1000, SEED_BASE + 1000 + TRAINING_PAIRS_MAX).
TRAINING_PAIRS_MAX = 8000


def train(F, t, steps: int = 2000, batch: int = 4096, lr: float = 1e-3, seed: int = 0, params=None, log=None):
    """Adam on the GPU kernels; returns (params, loss history)."""
    torch = _torch()
    N = F.shape[0]
    if params is None:
        params = torch.as_tensor(inputs.mlp_init_params(seed), device="cuda")
    params = params.clone()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.empty_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(seed + 1)
    hist = []
    for step in range(1, steps + 1):
        idx = torch.as_tensor(rng.integers(0, N, size=min(batch, N)), device="cuda")
        Fb = F[idx].contiguous()
        tb = t[idx].contiguous()
        goat.mlp_backward(Fb, tb, params, grad, loss)
        goat.mlp_adam(grad, params, m, v, step, lr)
        if step % 100 == 0 or step == 1:
            hist.append((step, float(loss.item())))
            if log:
                log(f"warmstart train step {step}: loss {hist[-1][1]:.4f}")
    return params, hist


def save(params, path: str = DEFAULT_PATH, meta: dict | None = None):
    from safetensors.numpy import save_file
    os.makedirs(os.path.dirname(path), exist_ok=True)
    arr = params.detach().cpu().numpy().astype(np.float32)
    save_file({"params": arr}, path, metadata={"layout": "W1[128][4],b1,W2[128][128],b2,W3[128],b3",
                                               "info": json.dumps(meta or {})})


def load(path: str = DEFAULT_PATH, device="cuda"):
    torch = _torch()
    from safetensors.numpy import load_file
    arr = load_file(path)["params"]
    if arr.shape[0] != goat.mlp_param_count():
        raise ValueError(f"{path}: {arr.shape[0]} parameters, expected {goat.mlp_param_count()}")
    return torch.as_tensor(arr, device=device)


def main(argv=None):
    """Generate samples with the plain solver, train on the GPU, save."""
    import argparse
    ap = argparse.ArgumentParser(description="train the Sinkhorn warm-start network")
    ap.add_argument("--pairs", type=int, default=TRAINING_PAIRS_MAX, help="pairs available to draw from")
    ap.add_argument("--solves", type=int, default=20000, help="stop generating after this many solves")
    ap.add_argument("--fw-iters", type=int, default=30)
    ap.add_argument("--workers", type=int, default=12, help="processes drawing the pairs")
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--out", default=DEFAULT_PATH)
    a = ap.parse_args(argv)
    if a.pairs > TRAINING_PAIRS_MAX:
        ap.error(f"--pairs must be at most {TRAINING_PAIRS_MAX} (held-out seeds follow)")

    def log(msg):
        print(msg, flush=True)

    t0 = time.time()
    pairs = training_pairs(a.pairs)
    F, t, meta = generate(pairs, fw_iters=a.fw_iters, log=log, max_solves=a.solves, workers=a.workers)
    used = len({m["seed"] for m in meta})
    log(f"{F.shape[0]} samples from {len(meta)} converged solves of {used} pairs ({time.time() - t0:.0f} s)")
    params, hist = train(F, t, steps=a.steps, batch=a.batch, lr=a.lr, seed=a.seed)
    log(f"loss {hist[0][1]:.4f} -> {hist[-1][1]:.4f} ({time.time() - t0:.0f} s)")
    save(params, a.out, meta=dict(pairs=used, fw_iters=a.fw_iters, steps=a.steps, batch=a.batch,
                                  lr=a.lr, seed=a.seed, samples=int(F.shape[0]), solves=len(meta),
                                  loss_first=hist[0][1], loss_last=hist[-1][1],
                                  seconds=round(time.time() - t0, 1)))
    log(f"saved {a.out}")


if __name__ == "__main__":
    main()
