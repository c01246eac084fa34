"""GPU parity of the learned warm start against the FP64 oracle
(oracle/mlp_oracle.py), and its use inside the solver."""
import numpy as np
import pytest

from oracle import goat_oracle as O
from oracle import mlp_oracle as M
from paper_2111_05366_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_05366_amd import goat
    goat.lib()
    yield goat
    goat.release_workspace()


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32), device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def unpack(vec):
    v = np.asarray(vec, np.float64)
    o = 0
    out = {}
    for k, shape in [("W1", (128, 4)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)),
                     ("W3", (1, 128)), ("b3", (1,))]:
        size = int(np.prod(shape))
        out[k] = v[o:o + size].reshape(shape)
        o += size
    assert o == v.size
    return out


def pack(d):
    return np.concatenate([d[k].reshape(-1) for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def _params(seed):
    p = I.mlp_init_params(seed)
    rng = np.random.default_rng(seed + 7)
    d = unpack(p)
    for k in ("b1", "b2", "b3"):
        d[k] = 0.1 * rng.normal(size=d[k].shape)
    return pack(d).astype(np.float32)


def _grad_problem(n, seed):
    g = I.rho_er_pair(n, min(0.5, 12.0 / n), 0.8, seed)
    U = I.uniform_matrix(n, seed + 1).astype(np.float64)
    P = 0.5 * (O.barycenter(n) + U / U.sum(axis=1, keepdims=True))
    return O.gradient(g.A.astype(float), g.B.astype(float), P).astype(np.float32)


def test_param_count(G):
    assert G.mlp_param_count() == 17281 == I.mlp_init_params(0).size


@pytest.mark.parametrize("n", [63, 257, 1000])
def test_features_parity(G, n):
    Gm = _grad_problem(n, 30 + n)
    eps = 0.03 * float(np.abs(Gm).max())
    F = host(G.mlp_features(dev(Gm), torch.tensor([eps], device="cuda")))
    ref = M.column_features(Gm.astype(np.float64), float(np.float32(eps)))
    scale = np.abs(ref).max(axis=0) + 1e-6
    err = np.max(np.abs(F - ref) / scale)
    print(f"features n={n}: max scaled err {err:.2e}")
    assert err <= 1e-4


def test_forward_backward_adam_parity(G):
    rng = np.random.default_rng(5)
    N = 1000
    F = rng.normal(size=(N, 4)).astype(np.float32)
    t = (np.sin(F[:, 0]) + 0.3 * F[:, 2]).astype(np.float32)
    p = _params(3)
    pd = unpack(p)
    y = host(G.mlp_forward(dev(F), dev(p)))
    yref, _ = M.forward(pd, F)
    assert np.max(np.abs(y - yref)) <= 1e-5 * (1 + np.max(np.abs(yref)))
    grad, loss = G.mlp_backward(dev(F), dev(t), dev(p))
    Lref, gref = M.loss_and_grads(pd, F, t)
    assert float(loss.item()) == pytest.approx(Lref, rel=1e-5)
    gd = unpack(host(grad))
    for k in gref:
        rel = np.linalg.norm(gd[k] - gref[k]) / max(np.linalg.norm(gref[k]), 1e-12)
        print(f"grad {k}: rel {rel:.2e}")
        assert rel <= 1e-4, k
    # one Adam step on the GPU vs the oracle's, from the same state
    P = dev(p)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    G.mlp_adam(grad, P, m, v, 1, 1e-3)
    pref = {k: val.copy() for k, val in pd.items()}
    mref = {k: np.zeros_like(val) for k, val in pd.items()}
    vref = {k: np.zeros_like(val) for k, val in pd.items()}
    M.adam_step(pref, gd, mref, vref, 1, 1e-3)
    assert np.max(np.abs(host(P) - pack(pref))) <= 1e-6


def test_backward_deterministic(G):
    rng = np.random.default_rng(6)
    F = dev(rng.normal(size=(777, 4)))
    t = dev(rng.normal(size=777))
    p = dev(_params(4))
    g1, _ = G.mlp_backward(F, t, p)
    g2, _ = G.mlp_backward(F, t, p)
    assert torch.equal(g1, g2)


def test_gpu_training_reduces_loss(G):
    from paper_2111_05366_amd import warmstart
    rng = np.random.default_rng(9)
    F = dev(rng.normal(size=(4096, 4)))
    t = torch.sin(F[:, 0]) + 0.5 * F[:, 3]
    params, hist = warmstart.train(F, t.contiguous(), steps=300, batch=1024, lr=3e-3, seed=2)
    assert hist[-1][1] < 0.2 * hist[0][1]


def test_solver_warm_modes_and_nan_fallback(G):
    g = I.rho_er_pair(150, 0.08, 0.9, 44)
    A, B = dev(g.A), dev(g.B)
    p = dev(_params(1))
    cold = G.solve(A, B, sk_max=400, fw_max=4, stop_on_stall=0)
    for warm in (1, 2, 3):
        r = G.solve(A, B, sk_max=400, fw_max=4, stop_on_stall=0, warm=warm, mlp_params=p)
        assert len(r.history) == 4
        # the start changes the path to the fixed point, not the fixed point:
        # the first direction agrees with the cold one when both converge
        if r.history[0]["sk_err"] <= 1e-6 and cold.history[0]["sk_err"] <= 1e-6:
            assert r.history[0]["c"] == pytest.approx(cold.history[0]["c"], rel=1e-5)
    bad = p.clone()
    bad[:10] = float("nan")
    r = G.solve(A, B, sk_max=400, fw_max=2, stop_on_stall=0, warm=2, mlp_params=bad)
    assert all(np.isfinite(h["fP"]) for h in r.history)
    with pytest.raises(G.GoatError):
        G.solve(A, B, warm=2)


def test_warm_start_same_fixed_point(G):
    n = 300
    Gm = _grad_problem(n, 71)
    Gd = dev(Gm)
    cold = G.sinkhorn(Gd, max_iter=5000, tol=1e-6)
    eps = cold.eps
    F = G.mlp_features(Gd, eps)
    pred = G.mlp_forward(F, dev(_params(2)))
    warm = G.sinkhorn(Gd, max_iter=5000, tol=1e-6, g0=(pred * eps).contiguous())
    assert float(cold.err.item()) <= 1e-6 and float(warm.err.item()) <= 1e-6
    assert np.max(np.abs(host(cold.Q) - host(warm.Q))) <= 1e-4


@pytest.mark.parametrize("n,iters", [(300, 5), (1000, 40), (2051, 12)])
def test_sinkhorn_network_start_parity(G, n, iters):
    """goat_sinkhorn with GOAT_INIT_MLP: the network's start evaluated in
    FP64 by the oracle from the same parameters, then the same number of
    sweeps, gives the same plan."""
    print(f"sinkhorn network start n={n} iters={iters}", flush=True)
    Gm = _grad_problem(n, 600 + n)
    params = _params(31)
    out = G.sinkhorn(dev(Gm), eps_rel=0.03, max_iter=iters, tol=0.0, mlp_params=dev(params))
    Gd = Gm.astype(np.float64)
    eps = 0.03 * float(np.max(np.abs(Gd)))
    assert float(out.eps.item()) == pytest.approx(eps, rel=1e-6)
    g0 = M.warm_start(Gd, eps, M.unpack(params))
    ref = O.log_sinkhorn_max(Gd, eps, tol=0.0, max_iter=iters, g0=g0)
    Qd = host(out.Q)
    err = float(np.linalg.norm(Qd - ref.Q) / np.linalg.norm(ref.Q))
    m = ref.Q >= 1e-30
    emax = float(np.max(np.abs(Qd[m] - ref.Q[m]) / ref.Q[m]))
    # the network's start is not the cold one: after one sweep the device
    # plan is the oracle's network-started plan, far from the cold-started one
    one = G.sinkhorn(dev(Gm), eps_rel=0.03, max_iter=1, tol=0.0, mlp_params=dev(params))
    ref1 = O.log_sinkhorn_max(Gd, eps, tol=0.0, max_iter=1, g0=g0)
    cold1 = O.log_sinkhorn_max(Gd, eps, tol=0.0, max_iter=1)
    Q1 = host(one.Q)
    sep = float(np.linalg.norm(cold1.Q - ref1.Q) / np.linalg.norm(ref1.Q))
    err1 = float(np.linalg.norm(Q1 - ref1.Q) / np.linalg.norm(ref1.Q))
    print(f"  Q rel_fro={err:.2e} elem={emax:.2e}; after one sweep {err1:.2e}, network vs cold start {sep:.2e}")
    assert err <= 1e-4 and emax <= 1e-4
    assert err1 <= 1e-4 and sep > 10 * err1
