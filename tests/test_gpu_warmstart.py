"""What the trained warm-start network gains over the solver without it.

The stored network (paper_2111_05366_amd/data/warmstart_mlp.safetensors,
written by ``python -m paper_2111_05366_amd.warmstart``) was trained on
correlated ER pairs with seeds disjoint from the held-out pairs below. On the
Sinkhorn problems of held-out Frank-Wolfe iterates it must reach the same
fixed point as the cold start in fewer iterations, and inside the solver it
must leave the final matching unchanged."""
import numpy as np
import pytest

from paper_2111_05366_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HELD_OUT = [(1200, 0.02, 0.7, I.SEED_BASE + 9001), (3000, 0.02, 0.7, I.SEED_BASE + 9002)]


@pytest.fixture(scope="module", autouse=True)
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_05366_amd import goat
    goat.lib()
    yield goat
    goat.release_workspace()


@pytest.fixture(scope="module")
def params(G):
    from paper_2111_05366_amd import warmstart
    return warmstart.load()


def test_training_seeds_disjoint_from_held_out():
    from paper_2111_05366_amd import warmstart
    train_seeds = {s for (_, _, _, s) in warmstart.training_pairs(warmstart.TRAINING_PAIRS_MAX)}
    assert not train_seeds & {s for (_, _, _, s) in HELD_OUT}


def test_stored_network_finite(G, params):
    assert params.numel() == G.mlp_param_count()
    assert bool(torch.isfinite(params).all())


def test_iterations_saved_on_held_out(G, params):
    cold_total = warm_total = lse_total = 0
    for (n, p, rho, seed) in HELD_OUT:
        g = I.rho_er_pair(n, p, rho, seed)
        A = torch.as_tensor(g.A, device="cuda")
        B = torch.as_tensor(g.B, device="cuda")
        run = G.Run(A, B, prec="fp32", sk_max=1000, stop_on_stall=1)
        rows = []
        for k in range(3):
            Gm = run.gradient()
            cold = G.sinkhorn(Gm, max_iter=3000, tol=1e-6)
            F = G.mlp_features(Gm, cold.eps)
            pred = G.mlp_forward(F, params)
            warm = G.sinkhorn(Gm, max_iter=3000, tol=1e-6, g0=(pred * cold.eps).contiguous())
            # baseline start: the first column update alone (the LSE feature)
            lse = G.sinkhorn(Gm, max_iter=3000, tol=1e-6, g0=(-F[:, 3] * cold.eps).contiguous(),
                             want_Q=False)
            # converged: the sweep's stop measure was within 1e-6; the error of
            # the returned plan is that measure recomputed from Q (FP32 sums in
            # another order), hence the 5 % margin
            for o in (cold, warm, lse):
                assert int(o.iters.item()) < 3000 and float(o.err.item()) <= 1.05e-6
            # same fixed point: Q agrees entrywise
            assert float((cold.Q - warm.Q).abs().max().item()) <= 1e-4 * float(cold.Q.abs().max().item())
            ic, iw, il = int(cold.iters.item()), int(warm.iters.item()), int(lse.iters.item())
            rows.append((ic, iw, il))
            cold_total += ic
            warm_total += iw
            lse_total += il
            if run.steps(1) == 0 or run.history[-1]["t"] == 0.0:
                break
        run.close()
        print(f"held-out n={n}: Sinkhorn iterations (cold, network, LSE start) per FW iterate {rows}")
    print(f"total: cold {cold_total}, network {warm_total}, LSE start {lse_total}")
    assert warm_total < cold_total
    assert warm_total < lse_total


def test_solver_with_network_keeps_matching(G, params):
    n, p, rho, seed = HELD_OUT[0]
    g = I.rho_er_pair(n, p, rho, seed)
    A = torch.as_tensor(g.A, device="cuda")
    B = torch.as_tensor(g.B, device="cuda")
    cold = G.solve(A, B, fw_max=8, sk_max=1000)
    net = G.solve(A, B, fw_max=8, sk_max=1000, warm=3, mlp_params=params)
    its_c = sum(h["sk_iters"] for h in cold.history)
    its_n = sum(h["sk_iters"] for h in net.history)
    mr_c = float(np.mean(cold.perm == g.truth))
    mr_n = float(np.mean(net.perm == g.truth))
    print("cold sk_iters", [h["sk_iters"] for h in cold.history],
          "network+previous sk_iters", [h["sk_iters"] for h in net.history])
    print(f"solver n={n}: Sinkhorn iterations cold {its_c}, network+previous {its_n}; "
          f"match ratio {mr_c:.4f} vs {mr_n:.4f}")
    assert its_n <= its_c
    assert abs(mr_n - mr_c) <= 0.005
